/*
 * oracle.c -- plain, slow, CPU reference evolver for a cosmic-string network.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. The product path (libsemipar) never
 * links, loads or calls it, and it shares no code with the HIP path.
 *
 * Everything is FP64, scalar, built with -ffp-contract=off (no fused multiply-add)
 * so that each expression below is evaluated exactly as written.
 *
 * What it computes (paper: Blanco-Pillado, Olum, Shlaer, "A new parallel simulation
 * technique", Section "Semi-parallel cosmic string simulation"):
 *
 *  - The string obeys the Nambu-Goto equation xdd = x'' in flat space, solved by
 *    x(sigma,t) = [a(t-sigma) + b(t+sigma)]/2 with piecewise-linear a and b; the world
 *    sheet is tiled by diamonds, each the sum of one a-piece and one b-piece, and in
 *    flat space every diamond is planar, so the lattice evolution is exact.
 *    Lattice form used here: one diamond at point k, step n, has bottom
 *    B = X[n-1][j], left L = X[n][k], right R = X[n][j] (j = next[k]) and top
 *    T = X[n+1][k] = L + (R - B)  (flat_top below).
 *  - In an expanding (flat Robertson-Walker) universe, comoving coordinates and
 *    conformal time are used and expansion enters at first order per diamond, so
 *    the future edges stay straight but are no longer parallel to the past edges.
 *    frw_top below is the first-order transport of both past edges across the
 *    diamond under the conformal-gauge FRW string equations, H = hcoef/eta.
 *  - Intersections between different pieces of string are searched each step and
 *    the two strings exchange partners with probability p (1 for field-theory
 *    strings; as low as 1e-3 for superstrings). Crossings that do not exchange
 *    partners pass through each other.
 *
 * Readings where the paper is silent (it defers these details to other papers):
 *  - "element" k of band n: the world-sheet strip between points k and next[k] from
 *    slice n to n+1, as two triangles U = (X[n][k], X[n][j], X[n+1][k]) and
 *    D = (X[n+1][k], X[n][j], X[n+1][j]).
 *  - "intersect": exact FP64 4-D bounding boxes overlap and one of the four
 *    triangle pairs has a solution of the 4x4 system by Cramer's rule inside both
 *    triangles (tri_tri below).
 *  - one event per element per step: events sorted by (t*, id_min, id_max) and
 *    accepted greedily.
 *  - exchange of partners: swap next[a] and next[b], fix prev.
 *  - probability p: every confirmed crossing of a step draws u in [0, 1) from the
 *    counter-based generator Philox4x64-10 (orc_philox4x64 below) with key
 *    (seed, 0) and counter (id_a, id_b, step, 0), u = (first output word >> 11) 2^-53,
 *    and exchanges partners only when u < p. The crossings that fail are logged
 *    (kind 1), claim no element, and count as events for loop removal; the greedy
 *    matching runs over the others.
 *  - periodic box of side L; positions unwrapped along each point's own trajectory;
 *    differences between distinct points use the minimum image L*rint(d/L).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_SURFACE (-2)
#define ORC_E_OOM (-3)

/* record flags */
#define FLAG_HAS_R 1  /* r, r_prev hold the right neighbour's vertices on slices step, step-1 */
#define FLAG_FROZEN 2 /* the point stopped in this region; (face + 1) << 8 names the face */
#define FLAG_ACTIVE 4 /* the point was still advancing when the evolution stopped */
#define FLAG_REMOVED 8 /* the point belongs to a loop that was recorded and removed */

typedef struct {
  int64_t id, next_id, prev_id;
  int32_t step, flags;
  double x[4], x_prev[4], r[4], r_prev[4];
} orc_rec;

typedef struct {
  int32_t step, kind;
  int64_t id_a, id_b;
  double t_star, x_star[3];
} orc_event;

typedef struct {
  double t;
  int64_t ida, idb;
  int64_t sa, sb;
  double x[3];
} orc_cand_event;

/* A loop recorded and removed: step, points, id of its lowest slot, energy, centre. */
typedef struct {
  int32_t step, n_points;
  int64_t rep_id;
  double energy, centre[3];
} orc_loop;

typedef struct {
  int64_t n;
  double L;
  int cosmology; /* 0 flat, 1 matter, 2 radiation (FRW with H = hcoef / eta) */
  double hcoef;
  int32_t step; /* slice index of cur */
  int64_t *id;
  int32_t *nx, *pv;
  double (*cur)[4], (*prv)[4], (*nw)[4];
  /* per element (band n) */
  double (*vert)[4][4];
  double (*lo)[4], (*hi)[4];
  /* event log */
  orc_event *log;
  int64_t nlog, caplog;
  /* bounded region (one 4-cube of the tiling); all fields unused when bounded == 0 */
  int bounded;
  double V[4];     /* lattice origin (x, y, z, tau) of the tiling */
  double inv2g;    /* 1 / (2 g), g the generator scale */
  double sqrt3;    /* tau = sqrt(3) t */
  int64_t idx[4];  /* region index */
  int32_t* fstep;  /* slice at which the point froze, INT32_MAX while active */
  int32_t* face;   /* face through which a frozen point's next diamond leaves */
  unsigned char *adv, *valid; /* advanced this step / element of this band exists */
  orc_rec* frz;    /* record captured when the point froze */
  int64_t n_active;
  /* confirmed events of the most recent step, in key order (for tests) */
  orc_cand_event *last_conf;
  int64_t n_last_conf;
  /* loop removal */
  int32_t step0;   /* slice of the initial surface */
  int32_t* ev;     /* step of the last logged event of each point's element */
  orc_loop* loops;
  int64_t nloops, caploops;
  /* intercommutation probability and the generator's seed */
  double p_ic;
  uint64_t seed;
  /* stats */
  int64_t point_steps, n_cand_total, n_conf_total, n_accepted_total, steps_done;
  int64_t n_passed_total;
} orc_region;

/* ------------------------------------------------------------------------------ */
/* Diamond tops                                                                     */
/* ------------------------------------------------------------------------------ */

/* Flat space, planar diamond: T = L + (R - B), component by component, this order. */
static void flat_top(const double Lp[4], const double Rp[4], const double Bp[4], double T[4]) {
  for (int c = 0; c < 4; ++c) T[c] = Lp[c] + (Rp[c] - Bp[c]);
}

/* Expanding universe, first order per diamond (conformal time eta = t).
 * With dL = L - B (spatial, minimum image), dR = R - B, alpha = t_L - t_B,
 * beta = t_R - t_B and H = hcoef / eta_m, eta_m = (t_L + t_R)/2:
 *   x_T = (x_L + dR) - H (beta dL + alpha dR)
 *   t_T = (t_L + beta) - H (alpha beta + dL.dR)
 * Derived from dp/deta = -H[q - (p.q)p] along the q-edge and dq/deta = -H[p - (p.q)q]
 * along the p-edge for the unit null directions p, q of the world sheet. */
static void frw_top(const double Lp[4], const double Rp[4], const double Bp[4], double box,
                    double hcoef, double T[4]) {
  double dL[3], dR[3];
  for (int c = 0; c < 3; ++c) {
    double d = Lp[c] - Bp[c];
    dL[c] = d - box * rint(d / box);
    dR[c] = Rp[c] - Bp[c];
  }
  double alpha = Lp[3] - Bp[3];
  double beta = Rp[3] - Bp[3];
  double eta_m = 0.5 * (Lp[3] + Rp[3]);
  double H = hcoef / eta_m;
  for (int c = 0; c < 3; ++c) {
    double hx = H * (beta * dL[c] + alpha * dR[c]);
    T[c] = (Lp[c] + dR[c]) - hx;
  }
  double dLdR = (dL[0] * dR[0] + dL[1] * dR[1]) + dL[2] * dR[2];
  T[3] = (Lp[3] + beta) - H * ((alpha * beta) + dLdR);
}

void orc_top(int cosmology, double hcoef, double box, const double Lp[4], const double Rp[4],
             const double Bp[4], double T[4]) {
  if (cosmology == 0)
    flat_top(Lp, Rp, Bp, T);
  else
    frw_top(Lp, Rp, Bp, box, hcoef, T);
}

/* ------------------------------------------------------------------------------ */
/* Counter-based random numbers                                                     */
/* ------------------------------------------------------------------------------ */

/* Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC 2011): ten rounds over a 4-word counter under a 2-word key. Each round
 * takes the two 128-bit products M0 c0 and M1 c2 and outputs
 * (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key grows by
 * the Weyl increments (W0, W1) before every round but the first. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* The uniform number of one crossing: u = (first word >> 11) 2^-53 in [0, 1). */
double orc_coin(uint64_t seed, int32_t step, int64_t id_a, int64_t id_b) {
  const uint64_t ctr[4] = {(uint64_t)id_a, (uint64_t)id_b, (uint64_t)(int64_t)step, 0};
  const uint64_t key[2] = {seed, 0};
  uint64_t o[4];
  orc_philox4x64(ctr, key, o);
  return (double)(o[0] >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------------------ */
/* Triangle-triangle intersection in 4-D                                            */
/* ------------------------------------------------------------------------------ */

/* 2x2 minors of rows (x,y) and (z,t). */
static double mxy(const double u[4], const double v[4]) { return u[0] * v[1] - u[1] * v[0]; }
static double mzt(const double u[4], const double v[4]) { return u[2] * v[3] - u[3] * v[2]; }

/* det[a b c d] (columns) by Laplace expansion along the row pairs (x,y) / (z,t). */
double orc_det4(const double a[4], const double b[4], const double c[4], const double d[4]) {
  double r = mxy(a, b) * mzt(c, d);
  r = r - mxy(a, c) * mzt(b, d);
  r = r + mxy(a, d) * mzt(b, c);
  r = r + mxy(b, c) * mzt(a, d);
  r = r - mxy(b, d) * mzt(a, c);
  r = r + mxy(c, d) * mzt(a, b);
  return r;
}

/* Triangles P0 + s E1 + u E2 and Q0 + v F1 + w F2. Solve
 * [E1 E2 (Q0-Q1) (Q0-Q2)] (s,u,v,w)^T = Q0 - P0 by Cramer's rule and accept when the
 * solution lies in both closed triangles and det != 0. Returns 1 on intersection and
 * the meeting point (X*, t*) computed on the P side. */
int orc_tri_tri(const double P0[4], const double P1[4], const double P2[4], const double Q0[4],
                const double Q1[4], const double Q2[4], double* t_out, double x_out[3]) {
  double E1[4], E2[4], G1[4], G2[4], D[4];
  for (int c = 0; c < 4; ++c) {
    E1[c] = P1[c] - P0[c];
    E2[c] = P2[c] - P0[c];
    G1[c] = Q0[c] - Q1[c];
    G2[c] = Q0[c] - Q2[c];
    D[c] = Q0[c] - P0[c];
  }
  double det = orc_det4(E1, E2, G1, G2);
  if (det == 0.0) return 0;
  double sn = orc_det4(D, E2, G1, G2);
  double un = orc_det4(E1, D, G1, G2);
  double vn = orc_det4(E1, E2, D, G2);
  double wn = orc_det4(E1, E2, G1, D);
  int ok;
  if (det > 0.0)
    ok = sn >= 0.0 && un >= 0.0 && (sn + un) <= det && vn >= 0.0 && wn >= 0.0 && (vn + wn) <= det;
  else
    ok = sn <= 0.0 && un <= 0.0 && (sn + un) >= det && vn <= 0.0 && wn <= 0.0 && (vn + wn) >= det;
  if (!ok) return 0;
  for (int c = 0; c < 3; ++c) x_out[c] = P0[c] + (sn * E1[c] + un * E2[c]) / det;
  *t_out = P0[3] + (sn * E1[3] + un * E2[3]) / det;
  return 1;
}

/* ------------------------------------------------------------------------------ */
/* Region                                                                           */
/* ------------------------------------------------------------------------------ */

typedef struct {
  int64_t id;
  int64_t slot;
} idslot;

static int cmp_idslot(const void* a, const void* b) {
  int64_t x = ((const idslot*)a)->id, y = ((const idslot*)b)->id;
  return (x > y) - (x < y);
}

static int64_t find_slot(const idslot* m, int64_t n, int64_t id) {
  int64_t lo = 0, hi = n - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (m[mid].id == id) return m[mid].slot;
    if (m[mid].id < id)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

void orc_destroy(orc_region* r) {
  if (!r) return;
  free(r->id);
  free(r->nx);
  free(r->pv);
  free(r->cur);
  free(r->prv);
  free(r->nw);
  free(r->vert);
  free(r->lo);
  free(r->hi);
  free(r->log);
  free(r->last_conf);
  free(r->fstep);
  free(r->face);
  free(r->adv);
  free(r->valid);
  free(r->frz);
  free(r->ev);
  free(r->loops);
  free(r);
}

/* Whole-volume region: every point must have both neighbours present and all records
 * must sit on the same slice. */
static int create_impl(const orc_rec* recs, int64_t n, double box, int cosmology, double hcoef,
                       int bounded, orc_region** out) {
  *out = NULL;
  if (n < 0 || !(box > 0.0)) return ORC_E_ARG;
  orc_region* r = (orc_region*)calloc(1, sizeof(orc_region));
  if (!r) return ORC_E_OOM;
  r->n = n;
  r->L = box;
  r->cosmology = cosmology;
  r->hcoef = hcoef;
  r->p_ic = 1.0;
  r->seed = 0;
  int64_t nn = n > 0 ? n : 1;
  r->id = (int64_t*)malloc(sizeof(int64_t) * nn);
  r->nx = (int32_t*)malloc(sizeof(int32_t) * nn);
  r->pv = (int32_t*)malloc(sizeof(int32_t) * nn);
  r->cur = malloc(sizeof(double[4]) * nn);
  r->prv = malloc(sizeof(double[4]) * nn);
  r->nw = malloc(sizeof(double[4]) * nn);
  r->vert = malloc(sizeof(double[4][4]) * nn);
  r->lo = malloc(sizeof(double[4]) * nn);
  r->hi = malloc(sizeof(double[4]) * nn);
  r->caplog = 1024;
  r->log = (orc_event*)malloc(sizeof(orc_event) * r->caplog);
  r->fstep = (int32_t*)malloc(sizeof(int32_t) * nn);
  r->face = (int32_t*)malloc(sizeof(int32_t) * nn);
  r->adv = (unsigned char*)malloc(nn);
  r->valid = (unsigned char*)malloc(nn);
  r->frz = (orc_rec*)calloc((size_t)nn, sizeof(orc_rec));
  r->ev = (int32_t*)malloc(sizeof(int32_t) * nn);
  idslot* map = (idslot*)malloc(sizeof(idslot) * nn);
  if (!r->id || !r->nx || !r->pv || !r->cur || !r->prv || !r->nw || !r->vert || !r->lo || !r->hi ||
      !r->log || !map || !r->fstep || !r->face || !r->adv || !r->valid || !r->frz || !r->ev) {
    free(map);
    orc_destroy(r);
    return ORC_E_OOM;
  }
  int rc = ORC_OK;
  for (int64_t k = 0; k < n; ++k) {
    map[k].id = recs[k].id;
    map[k].slot = k;
    r->id[k] = recs[k].id;
    memcpy(r->cur[k], recs[k].x, sizeof(double[4]));
    memcpy(r->prv[k], recs[k].x_prev, sizeof(double[4]));
    if (recs[k].step != recs[0].step) rc = ORC_E_SURFACE;
  }
  r->step = n > 0 ? recs[0].step : 1;
  r->step0 = r->step;
  /* no event yet: as if the last one were in the step before the initial slice */
  for (int64_t k = 0; k < n; ++k) r->ev[k] = r->step0 - 1;
  qsort(map, (size_t)n, sizeof(idslot), cmp_idslot);
  for (int64_t k = 1; k < n; ++k)
    if (map[k].id == map[k - 1].id) rc = ORC_E_SURFACE;
  for (int64_t k = 0; k < n && rc == ORC_OK; ++k) {
    int64_t a = recs[k].next_id < 0 ? -1 : find_slot(map, n, recs[k].next_id);
    int64_t b = recs[k].prev_id < 0 ? -1 : find_slot(map, n, recs[k].prev_id);
    if (!bounded && (a < 0 || b < 0)) rc = ORC_E_SURFACE;
    r->nx[k] = (int32_t)a;
    r->pv[k] = (int32_t)b;
    r->fstep[k] = INT32_MAX;
    r->face[k] = -1;
  }
  for (int64_t k = 0; k < n && rc == ORC_OK; ++k) {
    if (r->nx[k] >= 0 && r->pv[r->nx[k]] != k) rc = ORC_E_SURFACE;
    if (r->pv[k] >= 0 && r->nx[r->pv[k]] != k) rc = ORC_E_SURFACE;
  }
  r->n_active = n;
  free(map);
  if (rc != ORC_OK) {
    orc_destroy(r);
    return rc;
  }
  *out = r;
  return ORC_OK;
}

int orc_create(const orc_rec* recs, int64_t n, double box, int cosmology, double hcoef,
               orc_region** out) {
  return create_impl(recs, n, box, cosmology, hcoef, 0, out);
}

/* One 4-cube region of the tiling (Section "Geometry"): generators
 * g/2 (1,1,1,1), g/2 (1,-1,-1,1), g/2 (-1,1,-1,1), g/2 (-1,-1,1,1) in (x, y, z, tau),
 * tau = sqrt(3) t (the time shrink that makes the faces null), lattice origin V,
 * region index idx. geom = {V[0..3], inv2g, idx[0..3]}. Links may dangle (-1). */
int orc_create_bounded(const orc_rec* recs, int64_t n, double box, int cosmology, double hcoef,
                       const double geom[9], orc_region** out) {
  int rc = create_impl(recs, n, box, cosmology, hcoef, 1, out);
  if (rc != ORC_OK) return rc;
  orc_region* r = *out;
  r->bounded = 1;
  for (int i = 0; i < 4; ++i) r->V[i] = geom[i];
  r->inv2g = geom[4];
  for (int i = 0; i < 4; ++i) r->idx[i] = (int64_t)geom[5 + i];
  r->sqrt3 = sqrt(3.0);
  return ORC_OK;
}

/* Generator coordinates c = H^T (P - V) / (2 g) of a spacetime point (x, y, z, t). */
static void gen_coords(const double V[4], double inv2g, const double P[4], double c[4]) {
  double dx = P[0] - V[0];
  double dy = P[1] - V[1];
  double dz = P[2] - V[2];
  double dtau = sqrt(3.0) * P[3] - V[3];
  double a = dx + dy, b = dz + dtau, cc = dx - dy, d = dtau - dz;
  c[0] = (a + b) * inv2g;
  c[1] = (cc + d) * inv2g;
  c[2] = (d - cc) * inv2g;
  c[3] = (b - a) * inv2g;
}

void orc_region_coords(const orc_region* r, const double P[4], double c[4]) {
  gen_coords(r->V, r->inv2g, P, c);
}

/* Region of each of n spacetime points in a periodic tiling (Section "Geometry",
 * subsection "Boundary conditions": the tiling repeats with the box). The region index
 * is i = floor(c); its layer is S = i0 + i1 + i2 + i3 (regions of one layer share their
 * starting time) and its past vertex lies at spatial position p g/2 with
 * p = i0 h0 + i1 h1 + i2 h2 + i3 h3, h_m the generators' spatial directions (1,1,1),
 * (1,-1,-1), (-1,1,-1), (-1,-1,1). A shift by the box L along one axis changes i by
 * M (+-1, +-1, -+1, -+1) with K = 4 M = 4 L / (2 g), which leaves S and p mod K
 * unchanged, so (S, key) with key = (px K + py) K + pz, p taken mod K, names the region
 * up to the box's periodicity. */
void orc_region_keys(const double V[4], double inv2g, int32_t K, const double* P, int64_t n,
                     int32_t* S, int32_t* key) {
  for (int64_t q = 0; q < n; ++q) {
    double c[4];
    gen_coords(V, inv2g, P + 4 * q, c);
    int64_t i[4];
    for (int m = 0; m < 4; ++m) i[m] = (int64_t)floor(c[m]);
    int64_t p[3] = {i[0] + i[1] - i[2] - i[3], i[0] - i[1] + i[2] - i[3],
                    i[0] - i[1] - i[2] + i[3]};
    for (int m = 0; m < 3; ++m) p[m] = ((p[m] % K) + K) % K;
    S[q] = (int32_t)(i[0] + i[1] + i[2] + i[3]);
    key[q] = (int32_t)((p[0] * K + p[1]) * K + p[2]);
  }
}

/* -1 when P lies in the region (floor(c) == idx); otherwise the first i with
 * floor(c_i) > idx_i (the final face crossed), else the first i with floor(c_i) != idx_i. */
static int exit_face(const orc_region* r, const double P[4]) {
  double c[4];
  orc_region_coords(r, P, c);
  int first_ne = -1;
  for (int i = 0; i < 4; ++i) {
    double f = floor(c[i]);
    if (f > (double)r->idx[i]) return i;
    if (f != (double)r->idx[i] && first_ne < 0) first_ne = i;
  }
  return first_ne;
}

static void freeze(orc_region* r, int64_t k, int face, int with_r) {
  orc_rec* f = &r->frz[k];
  int64_t j = r->nx[k];
  memset(f, 0, sizeof(*f));
  f->id = r->id[k];
  f->next_id = j >= 0 ? r->id[j] : -1;
  f->prev_id = r->pv[k] >= 0 ? r->id[r->pv[k]] : -1;
  f->step = r->step;
  f->flags = FLAG_FROZEN | (with_r ? FLAG_HAS_R : 0) | ((face + 1) << 8);
  memcpy(f->x, r->cur[k], sizeof(double[4]));
  memcpy(f->x_prev, r->prv[k], sizeof(double[4]));
  if (with_r) {
    memcpy(f->r, r->cur[j], sizeof(double[4]));
    memcpy(f->r_prev, r->prv[j], sizeof(double[4]));
  }
}

/* Vertices and FP64 4-D bounding box of element k of the current band. */
static void build_element(orc_region* r, int64_t k) {
  int64_t j = r->nx[k];
  double sj[3];
  for (int c = 0; c < 3; ++c) sj[c] = r->L * rint((r->cur[j][c] - r->cur[k][c]) / r->L);
  double(*v)[4] = r->vert[k];
  for (int c = 0; c < 4; ++c) {
    double s = c < 3 ? sj[c] : 0.0;
    v[0][c] = r->cur[k][c];
    v[1][c] = c < 3 ? r->cur[j][c] - s : r->cur[j][c];
    v[2][c] = r->nw[k][c];
    v[3][c] = c < 3 ? r->nw[j][c] - s : r->nw[j][c];
  }
  for (int c = 0; c < 4; ++c) {
    double lo = v[0][c], hi = v[0][c];
    for (int i = 1; i < 4; ++i) {
      if (v[i][c] < lo) lo = v[i][c];
      if (v[i][c] > hi) hi = v[i][c];
    }
    r->lo[k][c] = lo;
    r->hi[k][c] = hi;
  }
}

/* Exact bounding-box overlap of elements a (id smaller) and b, b shifted onto a's
 * periodic image. */
static int pair_overlap(const orc_region* r, int64_t a, int64_t b, double S[3]) {
  for (int c = 0; c < 3; ++c) S[c] = r->L * rint((r->cur[b][c] - r->cur[a][c]) / r->L);
  for (int c = 0; c < 3; ++c) {
    if (!(r->lo[a][c] <= r->hi[b][c] - S[c])) return 0;
    if (!(r->lo[b][c] - S[c] <= r->hi[a][c])) return 0;
  }
  if (!(r->lo[a][3] <= r->hi[b][3])) return 0;
  if (!(r->lo[b][3] <= r->hi[a][3])) return 0;
  return 1;
}

static int is_adjacent(const orc_region* r, int64_t k, int64_t m) {
  return m == k || m == r->nx[k] || m == r->pv[k];
}

/* Test one candidate pair with all four triangle pairs; keep the smallest (t*, index). */
static int confirm_pair(const orc_region* r, int64_t k, int64_t m, orc_cand_event* ev) {
  int64_t a = k, b = m;
  if (r->id[b] < r->id[a]) {
    a = m;
    b = k;
  }
  double S[3];
  if (!pair_overlap(r, a, b, S)) return 0;
  double wb[4][4];
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 4; ++c) wb[i][c] = c < 3 ? r->vert[b][i][c] - S[c] : r->vert[b][i][c];
  const double(*va)[4] = (const double(*)[4])r->vert[a];
  /* U = (v0, v1, v2), D = (v2, v1, v3) */
  const double* Pa[2][3] = {{va[0], va[1], va[2]}, {va[2], va[1], va[3]}};
  const double* Qb[2][3] = {{wb[0], wb[1], wb[2]}, {wb[2], wb[1], wb[3]}};
  int found = 0;
  double bt = 0.0, bx[3] = {0, 0, 0};
  for (int ip = 0; ip < 2; ++ip)
    for (int iq = 0; iq < 2; ++iq) {
      double t, x[3];
      if (orc_tri_tri(Pa[ip][0], Pa[ip][1], Pa[ip][2], Qb[iq][0], Qb[iq][1], Qb[iq][2], &t, x)) {
        if (!found || t < bt) {
          found = 1;
          bt = t;
          bx[0] = x[0];
          bx[1] = x[1];
          bx[2] = x[2];
        }
      }
    }
  if (!found) return 0;
  ev->t = bt;
  ev->ida = r->id[a];
  ev->idb = r->id[b];
  ev->sa = a;
  ev->sb = b;
  memcpy(ev->x, bx, sizeof(bx));
  return 1;
}

static int cmp_event(const void* pa, const void* pb) {
  const orc_cand_event* a = (const orc_cand_event*)pa;
  const orc_cand_event* b = (const orc_cand_event*)pb;
  if (a->t < b->t) return -1;
  if (a->t > b->t) return 1;
  if (a->ida != b->ida) return a->ida < b->ida ? -1 : 1;
  if (a->idb != b->idb) return a->idb < b->idb ? -1 : 1;
  return 0;
}

typedef struct {
  int64_t* p;
  int64_t n, cap;
} pairvec;

static int pv_push(pairvec* v, int64_t a, int64_t b) {
  if (v->n + 1 > v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 1024;
    int64_t* np = (int64_t*)realloc(v->p, sizeof(int64_t) * 2 * nc);
    if (!np) return ORC_E_OOM;
    v->p = np;
    v->cap = nc;
  }
  v->p[2 * v->n] = a;
  v->p[2 * v->n + 1] = b;
  v->n++;
  return ORC_OK;
}

/* All pairs of non-adjacent elements with overlapping exact bounding boxes, by
 * brute force over every pair. */
static int search_brute(orc_region* r, pairvec* out) {
  double S[3];
  for (int64_t k = 0; k < r->n; ++k)
    for (int64_t m = k + 1; m < r->n; ++m) {
      if (!r->valid[k] || !r->valid[m] || is_adjacent(r, k, m)) continue;
      int64_t a = k, b = m;
      if (r->id[b] < r->id[a]) {
        a = m;
        b = k;
      }
      if (pair_overlap(r, a, b, S))
        if (pv_push(out, k, m)) return ORC_E_OOM;
    }
  return ORC_OK;
}

/* Bucket of cell (x, y, z) of the grid: a hash of the three coordinates, so that a
 * fine grid over a large box needs only as many buckets as there are elements. */
static uint64_t cell_bucket(int64_t x, int64_t y, int64_t z, uint64_t mask) {
  uint64_t h = (uint64_t)x * 0x9E3779B97F4A7C15ull;
  h ^= (uint64_t)y * 0xC2B2AE3D27D4EB4Full;
  h ^= (uint64_t)z * 0x165667B19E3779F9ull;
  h ^= h >> 29;
  return h & mask;
}

/* The same set through a uniform periodic grid whose cell is at least the largest
 * element extent: overlapping boxes then sit in neighbouring cells. Cells are hashed
 * into a power-of-two number of buckets (at least 2n); a bucket may hold elements of
 * several cells, which only adds pairs that the exact box test then rejects. Each
 * element visits the distinct buckets of its 27 neighbour cells once, and a pair is
 * taken from its element of lower slot, so every pair is tested at most once. */
static int search_grid(orc_region* r, pairvec* out) {
  int64_t n = r->n;
  double E = 0.0, maxabs = r->L;
  for (int64_t k = 0; k < n; ++k)
    for (int c = 0; c < 3 && r->valid[k]; ++c) {
      double e = r->hi[k][c] - r->lo[k][c];
      if (e > E) E = e;
      if (fabs(r->lo[k][c]) > maxabs) maxabs = fabs(r->lo[k][c]);
      if (fabs(r->hi[k][c]) > maxabs) maxabs = fabs(r->hi[k][c]);
    }
  double hmin = E + maxabs * 0x1p-36;
  double ncd = floor(r->L / hmin);
  if (ncd > 1024) ncd = 1024;
  if (ncd < 3) return search_brute(r, out);
  int64_t nc = (int64_t)ncd;
  double h = r->L / (double)nc;
  uint64_t nb = 1024;
  while (nb < 2 * (uint64_t)n) nb <<= 1;
  const uint64_t mask = nb - 1;
  int32_t(*cc)[3] = malloc(sizeof(int32_t[3]) * (n > 0 ? n : 1));
  uint64_t* bk = (uint64_t*)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
  int64_t* start = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
  int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  int64_t* fill = (int64_t*)calloc((size_t)nb, sizeof(int64_t));
  if (!cc || !bk || !start || !list || !fill) {
    free(cc);
    free(bk);
    free(start);
    free(list);
    free(fill);
    return ORC_E_OOM;
  }
  for (int64_t k = 0; k < n; ++k) {
    if (!r->valid[k]) {
      cc[k][0] = -1;
      continue;
    }
    for (int c = 0; c < 3; ++c) {
      double w = r->lo[k][c] - r->L * floor(r->lo[k][c] / r->L);
      int64_t ci = (int64_t)floor(w / h);
      if (ci < 0) ci = 0;
      if (ci > nc - 1) ci = nc - 1;
      cc[k][c] = (int32_t)ci;
    }
    bk[k] = cell_bucket(cc[k][0], cc[k][1], cc[k][2], mask);
    start[bk[k] + 1]++;
  }
  for (uint64_t i = 0; i < nb; ++i) start[i + 1] += start[i];
  for (int64_t k = 0; k < n; ++k) {
    if (cc[k][0] < 0) continue;
    list[start[bk[k]] + fill[bk[k]]++] = k;
  }
  int rc = ORC_OK;
  double S[3];
  for (int64_t k = 0; k < n && rc == ORC_OK; ++k) {
    if (cc[k][0] < 0) continue;
    uint64_t seen[27];
    int nseen = 0;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t x = (cc[k][0] + dx + nc) % nc, y = (cc[k][1] + dy + nc) % nc,
                  z = (cc[k][2] + dz + nc) % nc;
          uint64_t b = cell_bucket(x, y, z, mask);
          int dup = 0;
          for (int i = 0; i < nseen; ++i) dup |= seen[i] == b;
          if (dup) continue;
          seen[nseen++] = b;
          for (int64_t q = start[b]; q < start[b + 1]; ++q) {
            int64_t m = list[q];
            if (m <= k || is_adjacent(r, k, m)) continue;
            int64_t a = k, b2 = m;
            if (r->id[b2] < r->id[a]) {
              a = m;
              b2 = k;
            }
            if (pair_overlap(r, a, b2, S))
              if (pv_push(out, k, m)) rc = ORC_E_OOM;
          }
        }
  }
  free(cc);
  free(bk);
  free(start);
  free(list);
  free(fill);
  return rc;
}

static int log_push(orc_region* r, const orc_event* e) {
  if (r->nlog + 1 > r->caplog) {
    int64_t nc = 2 * r->caplog;
    orc_event* nl = (orc_event*)realloc(r->log, sizeof(orc_event) * nc);
    if (!nl) return ORC_E_OOM;
    r->log = nl;
    r->caplog = nc;
  }
  r->log[r->nlog++] = *e;
  return ORC_OK;
}

static int cmp_pair(const void* pa, const void* pb) {
  const int64_t* a = (const int64_t*)pa;
  const int64_t* b = (const int64_t*)pb;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

/* One lattice step: tops, elements, search, confirm, resolve, reconnect.
 * intercommute = 0 skips the intersection search (pure evolution). */
static int one_step(orc_region* r, int search, int intercommute) {
  int64_t n = r->n;
  int rc = ORC_OK;
  /* Which points advance. A bounded region computes the diamond of point k at step n
   * only when its earliest point, the bottom B = X[n-1][next[k]], lies in the region
   * (Section "Semi-parallel cosmic string simulation": each diamond is created in the
   * region that contains its earliest point) and both inputs exist; otherwise k stops
   * here and is handed on. All decisions use the state before the step. */
  if (r->bounded) {
    int32_t* nf = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t* nface = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    if (!nf || !nface) {
      free(nf);
      free(nface);
      return ORC_E_OOM;
    }
    for (int64_t k = 0; k < n; ++k) {
      nf[k] = r->fstep[k];
      nface[k] = r->face[k];
      r->adv[k] = 0;
      if (r->fstep[k] != INT32_MAX) continue;
      int64_t j = r->nx[k];
      if (j < 0) {
        freeze(r, k, -1, 0);
      } else if (r->fstep[j] < r->step) {
        freeze(r, k, r->face[j], 0);
      } else {
        int f = exit_face(r, r->prv[j]);
        if (f < 0) {
          r->adv[k] = 1;
          continue;
        }
        freeze(r, k, f, 1);
        nface[k] = f;
        nf[k] = r->step;
        continue;
      }
      nface[k] = j < 0 ? -1 : r->face[j];
      nf[k] = r->step;
    }
    for (int64_t k = 0; k < n; ++k) {
      if (nf[k] != r->fstep[k]) r->n_active--;
      r->fstep[k] = nf[k];
      r->face[k] = nface[k];
    }
    free(nf);
    free(nface);
  } else {
    for (int64_t k = 0; k < n; ++k) r->adv[k] = r->fstep[k] == INT32_MAX;
  }
  int64_t n_adv = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_adv)
  for (int64_t k = 0; k < n; ++k) {
    if (!r->adv[k]) continue;
    int64_t j = r->nx[k];
    orc_top(r->cosmology, r->hcoef, r->L, r->cur[k], r->cur[j], r->prv[j], r->nw[k]);
    n_adv++;
  }
  for (int64_t k = 0; k < n; ++k) r->valid[k] = r->adv[k] && r->nx[k] >= 0 && r->adv[r->nx[k]];
  if (!intercommute) goto rotate;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k)
    if (r->valid[k]) build_element(r, k);

  pairvec cand = {0, 0, 0};
  rc = search ? search_brute(r, &cand) : search_grid(r, &cand);
  if (rc != ORC_OK) {
    free(cand.p);
    return rc;
  }
  r->n_cand_total += cand.n;
  orc_cand_event* ev = (orc_cand_event*)malloc(sizeof(orc_cand_event) * (cand.n > 0 ? cand.n : 1));
  if (!ev) {
    free(cand.p);
    return ORC_E_OOM;
  }
  int64_t nev = 0;
  for (int64_t i = 0; i < cand.n; ++i)
    if (confirm_pair(r, cand.p[2 * i], cand.p[2 * i + 1], &ev[nev])) nev++;
  free(cand.p);
  r->n_conf_total += nev;
  qsort(ev, (size_t)nev, sizeof(orc_cand_event), cmp_event);
  free(r->last_conf);
  r->last_conf = (orc_cand_event*)malloc(sizeof(orc_cand_event) * (nev > 0 ? nev : 1));
  if (r->last_conf) memcpy(r->last_conf, ev, sizeof(orc_cand_event) * (size_t)nev);
  r->n_last_conf = r->last_conf ? nev : 0;

  /* greedy: one event per element per step */
  unsigned char* used = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
  if (!used) {
    free(ev);
    return ORC_E_OOM;
  }
  for (int64_t i = 0; i < nev && rc == ORC_OK; ++i) {
    int64_t a = ev[i].sa, b = ev[i].sb;
    if (!(orc_coin(r->seed, r->step, ev[i].ida, ev[i].idb) < r->p_ic)) {
      /* the strings pass through each other: logged, no exchange, no claim */
      r->ev[a] = r->ev[b] = r->step;
      orc_event e;
      e.step = r->step;
      e.kind = 1;
      e.id_a = ev[i].ida;
      e.id_b = ev[i].idb;
      e.t_star = ev[i].t;
      memcpy(e.x_star, ev[i].x, sizeof(e.x_star));
      rc = log_push(r, &e);
      r->n_passed_total++;
      continue;
    }
    if (used[a] || used[b]) continue;
    used[a] = used[b] = 1;
    int32_t ja = r->nx[a], jb = r->nx[b];
    r->nx[a] = jb;
    r->nx[b] = ja;
    r->pv[jb] = (int32_t)a;
    r->pv[ja] = (int32_t)b;
    r->ev[a] = r->ev[b] = r->step;
    orc_event e;
    e.step = r->step;
    e.kind = 0;
    e.id_a = ev[i].ida;
    e.id_b = ev[i].idb;
    e.t_star = ev[i].t;
    memcpy(e.x_star, ev[i].x, sizeof(e.x_star));
    rc = log_push(r, &e);
    r->n_accepted_total++;
  }
  free(used);
  free(ev);

rotate:;
  double(*tmp)[4] = r->prv;
  r->prv = r->cur;
  r->cur = r->nw;
  r->nw = tmp;
  r->step += 1;
  r->point_steps += n_adv;
  r->steps_done += 1;
  return rc;
}

/* Loop record and removal (Section "Semi-parallel cosmic string simulation": loops that
 * will not intersect again are recorded and removed). Reading: at the start of a step
 * n, a closed chain of still-active points (a loop) of L points is removed when no
 * logged event (an exchange, or with p < 1 a crossing that passed through) touched
 * any of its elements during the last L steps, n - L .. n - 1
 * (its period in flat space), and every point lies within a quarter of the box, per
 * axis, of the loop's lowest slot (a string winding the box never does). The record holds the step, L, the
 * id of the lowest slot, the energy sum over k of |X[n][k] - X[n-1][j]| + |X[n][j] -
 * X[n-1][j]| (j = next k; spatial, minimum image) and the centre, the mean position
 * about the lowest slot. The loop's points stop (flag REMOVED, no owning face). */
static int loop_check(orc_region* r) {
  int64_t n = r->n;
  unsigned char* seen = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
  int64_t* cyc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!seen || !cyc) {
    free(seen);
    free(cyc);
    return ORC_E_OOM;
  }
  int rc = ORC_OK;
  for (int64_t k0 = 0; k0 < n && rc == ORC_OK; ++k0) {
    if (seen[k0] || r->fstep[k0] != INT32_MAX) continue;
    /* walk forward from k0: a loop when it returns to k0 through unseen active points */
    int64_t L = 0, k = k0;
    int closed = 0;
    for (;;) {
      if (k < 0 || seen[k] || r->fstep[k] != INT32_MAX) break;
      seen[k] = 1;
      cyc[L++] = k;
      k = r->nx[k];
      if (k == k0) {
        closed = 1;
        break;
      }
    }
    if (!closed) continue;
    int64_t rep = cyc[0];
    int32_t last = r->step0 - 1;
    for (int64_t i = 0; i < L; ++i) {
      if (cyc[i] < rep) rep = cyc[i];
      if (r->ev[cyc[i]] > last) last = r->ev[cyc[i]];
    }
    /* an event in step e changes the loop from step e + 1 on: quiet for a full period
     * when the steps e + 1 .. e + L have all been taken, n > e + L */
    if ((int64_t)r->step - last <= L) continue;
    int compact = 1;
    for (int64_t i = 0; i < L && compact; ++i)
      for (int c = 0; c < 3; ++c) {
        double d = r->cur[cyc[i]][c] - r->cur[rep][c];
        d -= r->L * rint(d / r->L);
        if (!(fabs(d) < 0.25 * r->L)) compact = 0;
      }
    if (!compact) continue;
    orc_loop lp;
    lp.step = r->step;
    lp.n_points = (int32_t)L;
    lp.rep_id = r->id[rep];
    double e = 0.0, cs[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < L; ++i) {
      int64_t a = cyc[i], j = r->nx[a];
      double da[3], db[3];
      for (int c = 0; c < 3; ++c) {
        da[c] = r->cur[a][c] - r->prv[j][c];
        da[c] -= r->L * rint(da[c] / r->L);
        db[c] = r->cur[j][c] - r->prv[j][c];
        double d = r->cur[a][c] - r->cur[rep][c];
        cs[c] += d - r->L * rint(d / r->L);
      }
      e += sqrt(da[0] * da[0] + da[1] * da[1] + da[2] * da[2]) +
           sqrt(db[0] * db[0] + db[1] * db[1] + db[2] * db[2]);
    }
    lp.energy = e;
    for (int c = 0; c < 3; ++c) lp.centre[c] = r->cur[rep][c] + cs[c] / (double)L;
    if (r->nloops == r->caploops) {
      int64_t nc = r->caploops ? 2 * r->caploops : 64;
      orc_loop* nl = (orc_loop*)realloc(r->loops, sizeof(orc_loop) * (size_t)nc);
      if (!nl) {
        rc = ORC_E_OOM;
        break;
      }
      r->loops = nl;
      r->caploops = nc;
    }
    r->loops[r->nloops++] = lp;
    for (int64_t i = 0; i < L; ++i) {
      int64_t a = cyc[i];
      orc_rec* f = &r->frz[a];
      memset(f, 0, sizeof(*f));
      f->id = r->id[a];
      f->next_id = r->id[r->nx[a]];
      f->prev_id = r->id[r->pv[a]];
      f->step = r->step;
      f->flags = FLAG_REMOVED;
      memcpy(f->x, r->cur[a], sizeof(double[4]));
      memcpy(f->x_prev, r->prv[a], sizeof(double[4]));
      r->fstep[a] = r->step;
      r->face[a] = -1;
      r->n_active--;
    }
  }
  free(seen);
  free(cyc);
  return rc;
}

int64_t orc_loop_count(const orc_region* r) { return r->nloops; }

int orc_loops(const orc_region* r, orc_loop* out) {
  if (r->nloops) memcpy(out, r->loops, sizeof(orc_loop) * (size_t)r->nloops);
  return ORC_OK;
}

/* Evolve until max_steps steps were taken, or until the smallest time on the current
 * slice reaches t_end. search: 0 = periodic grid, 1 = brute force over all pairs.
 * loop_every > 0: loop record and removal before every step n with n - step0 a
 * positive multiple of loop_every. */
int orc_evolve(orc_region* r, int64_t max_steps, double t_end, int search, int intercommute,
               int32_t loop_every) {
  if (!r || loop_every < 0) return ORC_E_ARG;
  for (int64_t s = 0; s < max_steps; ++s) {
    if (r->n_active == 0) break;
    if (loop_every > 0 && r->step > r->step0 && (r->step - r->step0) % loop_every == 0) {
      int rc = loop_check(r);
      if (rc != ORC_OK) return rc;
      if (r->n_active == 0) break;
    }
    double tmin = INFINITY;
    for (int64_t k = 0; k < r->n; ++k)
      if (r->fstep[k] == INT32_MAX && r->cur[k][3] < tmin) tmin = r->cur[k][3];
    if (tmin >= t_end) break;
    int rc = one_step(r, search, intercommute);
    if (rc != ORC_OK) return rc;
  }
  return ORC_OK;
}

/* Candidate set of the current band without advancing (pairs of ids, id_a < id_b,
 * sorted). Returns the count; writes at most cap pairs. */
int64_t orc_band_candidates(orc_region* r, int search, int64_t* out, int64_t cap) {
  int64_t n = r->n;
  for (int64_t k = 0; k < n; ++k) r->valid[k] = 1;
  for (int64_t k = 0; k < n; ++k) {
    int64_t j = r->nx[k];
    orc_top(r->cosmology, r->hcoef, r->L, r->cur[k], r->cur[j], r->prv[j], r->nw[k]);
  }
  for (int64_t k = 0; k < n; ++k) build_element(r, k);
  pairvec cand = {0, 0, 0};
  int rc = search ? search_brute(r, &cand) : search_grid(r, &cand);
  if (rc != ORC_OK) {
    free(cand.p);
    return rc;
  }
  for (int64_t i = 0; i < cand.n; ++i) {
    int64_t a = r->id[cand.p[2 * i]], b = r->id[cand.p[2 * i + 1]];
    cand.p[2 * i] = a < b ? a : b;
    cand.p[2 * i + 1] = a < b ? b : a;
  }
  qsort(cand.p, (size_t)cand.n, 2 * sizeof(int64_t), cmp_pair);
  int64_t m = cand.n < cap ? cand.n : cap;
  if (out) memcpy(out, cand.p, sizeof(int64_t) * 2 * m);
  int64_t total = cand.n;
  free(cand.p);
  return total;
}

/* Confirmed events of the most recent step (sorted by key), as (t, ida, idb, x). */
int64_t orc_last_confirmed(const orc_region* r, double* t, int64_t* ids, double* x) {
  for (int64_t i = 0; i < r->n_last_conf; ++i) {
    if (t) t[i] = r->last_conf[i].t;
    if (ids) {
      ids[2 * i] = r->last_conf[i].ida;
      ids[2 * i + 1] = r->last_conf[i].idb;
    }
    if (x) memcpy(&x[3 * i], r->last_conf[i].x, sizeof(double[3]));
  }
  return r->n_last_conf;
}

int64_t orc_n(const orc_region* r) { return r->n; }
int64_t orc_active(const orc_region* r) { return r->n_active; }
int32_t orc_step(const orc_region* r) { return r->step; }
int64_t orc_event_count(const orc_region* r) { return r->nlog; }

void orc_stats(const orc_region* r, int64_t out[6]) {
  out[0] = r->point_steps;
  out[1] = r->n_cand_total;
  out[2] = r->n_conf_total;
  out[3] = r->n_accepted_total;
  out[4] = r->steps_done;
  out[5] = r->n_passed_total;
}

/* Intercommutation probability p in [0, 1] and the generator's seed for later steps
 * (the default is p = 1: every accepted crossing exchanges partners; p = 0: every
 * crossing passes through, so the network's links never change). */
int orc_set_coin(orc_region* r, double p, uint64_t seed) {
  if (!r || !(p >= 0.0 && p <= 1.0)) return ORC_E_ARG;
  r->p_ic = p;
  r->seed = seed;
  return ORC_OK;
}

int orc_events(const orc_region* r, orc_event* out) {
  memcpy(out, r->log, sizeof(orc_event) * (size_t)r->nlog);
  return ORC_OK;
}

/* Current state as records in slot order: x = slice step, x_prev = slice step-1. */
int orc_read(const orc_region* r, orc_rec* out) {
  for (int64_t k = 0; k < r->n; ++k) {
    if (r->fstep[k] != INT32_MAX) {
      out[k] = r->frz[k];
      continue;
    }
    memset(&out[k], 0, sizeof(orc_rec));
    if (r->bounded) out[k].flags = FLAG_ACTIVE;
    out[k].id = r->id[k];
    out[k].next_id = r->nx[k] >= 0 ? r->id[r->nx[k]] : -1;
    out[k].prev_id = r->pv[k] >= 0 ? r->id[r->pv[k]] : -1;
    out[k].step = r->step;
    memcpy(out[k].x, r->cur[k], sizeof(double[4]));
    memcpy(out[k].x_prev, r->prv[k], sizeof(double[4]));
  }
  return ORC_OK;
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
