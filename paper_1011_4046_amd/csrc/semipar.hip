// semipar.hip -- libsemipar: evolution of one globally hyperbolic region of a
// cosmic-string network on an MI355X (gfx950).
//
// Paper: Blanco-Pillado, Olum, Shlaer, "A new parallel simulation technique",
// Section "Semi-parallel cosmic string simulation": construct all diamonds of the
// world sheet, look for intersections between different pieces of string, and
// reconnect the strings at the intersections.
//
// One lattice step n of a whole-volume region is six kernels on one stream:
//   k_evolve      diamond tops X[n+1] (flat or first-order FRW) fused with the
//                 element of band n (vertices, FP64 box, cell, bucket count)
//   k_scan        exclusive scan of bucket counts (counts reset to 0)
//   k_scatter     cell-sorted copies of element cell, slot and screen box
//   k_screen      half-shell bounding-box screen (FP64 or FP32) -> candidate pairs
//   k_confirm     exact FP64 box overlap + four triangle pairs -> events
//   k_resolve     one event per element by iterated local minima of (t*, id_a, id_b),
//                 partner exchange, event log, step bookkeeping (one workgroup)
// A device control block carries the step index, the stop rule and the counters,
// so a block of steps can be issued (or graph-replayed) without host round trips.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <new>
#include <type_traits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "semipar.h"
#include "geom.h"
#include "internal.h"

#pragma clang fp contract(off)

using sp::Box4;
using sp::Elem;
using sp::V4;

namespace {

constexpr int TS_LOG = 12;  // buckets per scan tile = 4096
constexpr int TS = 1 << TS_LOG;
constexpr int NT = 256;        // threads per block of the per-point kernels
constexpr int RESOLVE_NT = 1024;
constexpr uint64_t KEY_MAX = ~0ull;

// ---------------------------------------------------------------------------------
// device data
// ---------------------------------------------------------------------------------
// Cell grid of the current step (chosen at the end of the previous step).
struct Cells {
  int32_t nc;      // cells per dimension (>= 3), 0 = every element is large
  int32_t fixed;   // 1: keep this grid; 0: follow the largest element of each step
  double h;        // cell edge = box / nc
  double inv_h;    // 1 / h
  double hlim;     // elements with a larger spatial extent are large
  float h32;       // h in FP32
  float marg32;    // slack of FP32 spatial comparisons
};

// One 4-cube of the spacetime tiling: generator coordinates c = H^T (P - V) / (2 g)
// with tau = sqrt(3) t, region = floor(c) == idx.
struct RegionGeom {
  double V[4];
  double inv2g;
  double sqrt3;
  int32_t idx[4];
};

// Spatial centre of the region: the lattice origin moved by the region's index along
// the generators, whose spatial parts are g/2 (1,1,1), (1,-1,-1), (-1,1,-1), (-1,-1,1).
// Every point of the region lies within g of it per axis.
__host__ __device__ inline void region_centre(const RegionGeom& G, double c[3]) {
  const double h = 0.25 / G.inv2g;  // g / 2
  const int a = G.idx[0], b = G.idx[1], e = G.idx[2], d = G.idx[3];
  c[0] = G.V[0] + h * (double)(a + b - e - d);
  c[1] = G.V[1] + h * (double)(a - b + e - d);
  c[2] = G.V[2] + h * (double)(a - b - e + d);
}

// -1 when P lies in the region; else the first i with floor(c_i) > idx_i (the final face
// its future leaves by), else the first i with floor(c_i) != idx_i.
__device__ __forceinline__ int exit_face(const RegionGeom& G, const V4& P) {
  const double dx = P.x - G.V[0];
  const double dy = P.y - G.V[1];
  const double dz = P.z - G.V[2];
  const double dtau = G.sqrt3 * P.t - G.V[3];
  const double a = dx + dy, b = dz + dtau, cc = dx - dy, d = dtau - dz;
  const double c[4] = {(a + b) * G.inv2g, (cc + d) * G.inv2g, (d - cc) * G.inv2g,
                       (b - a) * G.inv2g};
  int first_ne = -1;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double f = floor(c[i]);
    if (f > (double)G.idx[i]) return i;
    if (f != (double)G.idx[i] && first_ne < 0) first_ne = i;
  }
  return first_ne;
}

constexpr int32_t FS_ACTIVE = INT32_MAX;  // stop step of a point that still advances
constexpr int32_t NO_ELEM = INT32_MIN;    // ecell of a point without an element this band

// Default cell edge of the next step, in units of this step's largest element extent
// (semipar_evolve_params.cell_factor overrides it): any value >= 1 gives the same
// candidates; larger cells hold more entries, smaller ones send more elements to the
// all-pairs path of large elements.
constexpr double CELL_GROW = 1.15;

struct Ctrl {
  int32_t step;        // lattice index of the current slice
  int32_t step_limit;  // a step is taken only while step < step_limit
  int32_t done;        // set: every kernel of a step returns at once
  int32_t defer;       // step not taken: 1 candidates, 2 events, 4 log overflowed
  int32_t stamp;       // resolve iteration stamp
  uint64_t tmin_key;   // order key of the smallest t of the slice being written
  double t_end;
  int64_t point_steps, cand_total, conf_total, acc_total, large_total, steps_taken;
  int64_t pass_total;  // crossings that passed through (probability p < 1)
  int64_t log_n;
  int64_t n_points;
  int64_t last_cand;   // candidate appends of the last step taken (may exceed the buffer)
  int32_t err;
  int32_t start_last;  // hand-off batch: the last step at which a point starts (else
                       // INT32_MIN): the batch is not done before it
  uint64_t ext_key;    // init: order key of an element-size estimate
  Cells cells;         // grid of the current step
  double box;          // periodic length (for the grid choice)
  double grow;         // next cell = grow * largest element extent of this step
  double tol;          // slack of FP64 spatial comparisons
  // the counters that the step kernels update atomically, on a cache line apart from
  // the fields every workgroup reads at its start
  alignas(128) int32_t n_cand;  // candidate appends this step (may exceed the buffer)
  int32_t n_evt;                // confirmed crossings this step (may exceed the buffer)
  int32_t n_large;              // elements of this step outside the hash
  // the event matching's workgroups: log places taken, exchanges, pass-throughs, most
  // rounds of a group, and workgroups finished (all zero between steps)
  int32_t res_nlog, res_nacc, res_npass, res_iter, res_done;
  int32_t pb_step;    // persistent launch: the furthest slice any of its regions reached
  int64_t tok_n;      // hand-off batch: start tokens written (may exceed the buffer)
  int32_t n_act;      // bounded region: entries of the list of advancing points
};

// The last three slices of every point, one 32-byte vertex (x, y, z, t) per point per
// slice: a gather through next[] then touches one 32-byte piece (two 16-byte loads), where
// four separate coordinate arrays took four loads from four cache lines.
struct Slices {
  double4* p[3];  // [slice mod 3][point]
};

struct EvCand {
  double t;
  int64_t ida, idb;
  int32_t sa, sb;
  double x, y, z;
};

struct LargeBox {
  double wl[3];   // wrapped lower corner
  double ext[3];  // extents
  double tlo, thi;
  int32_t slot;
  int32_t pad;
};

struct HashCfg {   // fixed for a configuration
  uint32_t bmask;  // buckets - 1
  int32_t B;       // buckets (power of two, >= TS)
  double tol;      // slack of FP64 spatial comparisons
  double tolL;     // slack of the large-element (wrapped) comparisons
  double tref;     // time origin of FP32 boxes
  double tol_t;    // slack of FP32 time conversion
};

// Local grid of one sub-region of a batch: a non-periodic cube of side W = 2.5 g around
// the region's spatial centre (the region's points lie within g of it per axis), nc^3
// cells of edge h. Elements outside are clamped into the boundary cells, which only
// merges cells (more pairs tested, never fewer). Cells of region q occupy the buckets
// (base + row-major index) mod B; cell keys carry the region's salt.
struct RCell {
  double ox, oy, oz;  // grid origin
  double h, inv_h, hlim;
  float h32, marg32;
  int32_t nc;
  uint32_t base;
  uint32_t salt;
  int32_t pad;
};
constexpr double RCELL_W = 2.5;  // grid side in units of g
// Per-sub-region extent maxima sit one cache line apart: every wave of a sub-region
// updates its entry each step, and neighbouring entries on one line would serialise the
// atomics of different sub-regions.
constexpr int REXT_STRIDE = 16;

// ---- hand-off between the regions of a tiling -------------------------------------
// A tiling run keeps the whole world sheet in device memory: the vertex of every point on
// every slice, written once by the region that builds the diamond with that top and read
// by every later region that needs it (Section "Semi-parallel cosmic string simulation":
// a diamond is built by the region that holds its earliest point, and what overlaps a
// region's final surfaces is passed on to its successors). A region's work list is a set
// of start tokens: point q builds its diamonds in region R from step n on, because its
// right neighbour's world line entered R at slice n - 1.
using spi::HandTok;

// Region names of the periodic tiling, the world sheet, and a hand-off batch's own
// per-point tables (passed by value to the step kernel of such a batch).
struct HistCfg {
  double4* H;             // [slice - s0][slot]; t = NaN: not built
  int64_t* home;          // [slice - s0][slot]: name of the vertex's home (HOME_NONE: not built)
  int64_t n;              // points of the volume
  int32_t s0, ns;         // first slice held, slices held
  double V[4];            // lattice origin (x, y, z, tau)
  double inv2g, sqrt3;
  int32_t K, S_lo, S_hi;  // names repeat with the box every K past-vertex steps
  int32_t pad;
  const int32_t* lut;     // [(S - S_lo) K^3 + key] -> region index, -1: not in the tiling
  const int64_t* sname;   // per sub-region of the batch: its region's name
  const int32_t* gnext;   // per volume slot: right neighbour's slot
  const int32_t* gprev;   // per volume slot: left neighbour's slot
  const int32_t* gsl;     // per local slot: volume slot
  const int32_t* gnx;     // per local slot: volume slot of its right neighbour
  const int32_t* start;   // per local slot: first step it builds a diamond here
  HandTok* tok;           // tokens for other regions (capacity tok_cap)
  int64_t tok_cap;
};

constexpr int32_t HERR_INPUT = 256;    // a diamond's input was never built
constexpr int32_t HERR_START = 512;    // a start token whose diamond is not the region's
constexpr int32_t HERR_SLICES = 1024;  // the world sheet holds too few slices
constexpr int32_t HERR_SELF = 2048;    // a world line re-entered the region building it
constexpr int32_t HERR_TOKENS = 4096;  // the token buffer overflowed
constexpr int32_t HERR_TIE = 8192;     // a diamond's inputs have two homes of one layer
constexpr int32_t HERR_MASK =
    HERR_INPUT | HERR_START | HERR_SLICES | HERR_SELF | HERR_TOKENS | HERR_TIE;
constexpr int64_t HOME_NONE = INT64_MIN;

// Name (S << 32 | key) of the region holding P: generator coordinates in the same
// arithmetic as exit_face, index i = floor(c), layer S = sum i, past vertex p g/2 with
// p = i0 h0 + i1 h1 + i2 h2 + i3 h3 (h_m the generators' spatial directions), key of
// p mod K. A shift by the box changes i by K/4 (+-1, +-1, -+1, -+1), which keeps both.
__device__ __forceinline__ int64_t hist_name(const HistCfg& h, const V4& P) {
  const double dx = P.x - h.V[0];
  const double dy = P.y - h.V[1];
  const double dz = P.z - h.V[2];
  const double dtau = h.sqrt3 * P.t - h.V[3];
  const double a = dx + dy, b = dz + dtau, cc = dx - dy, d = dtau - dz;
  const int i0 = (int)floor((a + b) * h.inv2g);
  const int i1 = (int)floor((cc + d) * h.inv2g);
  const int i2 = (int)floor((d - cc) * h.inv2g);
  const int i3 = (int)floor((b - a) * h.inv2g);
  const int K = h.K;
  int px = (i0 + i1 - i2 - i3) % K, py = (i0 - i1 + i2 - i3) % K, pz = (i0 - i1 - i2 + i3) % K;
  px += px < 0 ? K : 0;
  py += py < 0 ? K : 0;
  pz += pz < 0 ? K : 0;
  const int S = i0 + i1 + i2 + i3;
  return ((int64_t)S << 32) | (int64_t)(uint32_t)((px * K + py) * K + pz);
}

__device__ __forceinline__ int32_t hist_region(const HistCfg& h, int64_t name) {
  const int S = (int)(name >> 32);
  const int key = (int)(uint32_t)(name & 0xffffffffll);
  if (S < h.S_lo || S > h.S_hi) return -1;
  return h.lut[(int64_t)(S - h.S_lo) * h.K * h.K * h.K + key];
}

// Home of a new vertex: the region holding it (name o), unless a vertex its diamond was
// built from has a home of a later layer -- the first-order expansion can leave an edge
// slightly outside the light cone, so that a world line steps back across a face --,
// then that later home. Two different homes of the latest layer set *tie.
__device__ __forceinline__ int64_t resolve_home(int64_t o, int64_t a, int64_t b, int64_t c,
                                                bool* tie) {
  int64_t m = a;
  m = (b >> 32) > (m >> 32) ? b : m;
  m = (c >> 32) > (m >> 32) ? c : m;
  const bool later = (o >> 32) > (m >> 32);
  if (!later) {
    const int64_t Sm = m >> 32;
    *tie = ((a >> 32) == Sm && a != m) || ((b >> 32) == Sm && b != m) ||
           ((c >> 32) == Sm && c != m);
  }
  return (o == m || later) ? o : m;
}

__device__ __forceinline__ int64_t ldhome(const HistCfg& h, int s, int g) {
  return h.home[(int64_t)(s - h.s0) * h.n + g];
}

__device__ __forceinline__ V4 ldh(const HistCfg& h, int s, int g) {
  const double4 v = h.H[(int64_t)(s - h.s0) * h.n + g];
  return V4{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ V4 ld(const Slices& X, int s, int k) {
  const double4 v = X.p[s][k];
  return V4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void st(const Slices& X, int s, int k, const V4& v) {
  X.p[s][k] = make_double4(v.x, v.y, v.z, v.t);
}

__host__ __device__ __forceinline__ uint64_t order_key(double v) {
  uint64_t b;
  memcpy(&b, &v, 8);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double from_key(uint64_t k) {
  uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  double v;
  memcpy(&v, &b, 8);
  return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// True when every active lane of the wave holds the same key (sub-region, chain) as lane 0.
__device__ __forceinline__ bool wave_uniform(int q, bool live) {
  const int q0 = __shfl(q, 0, 64);
  const uint64_t live_m = __ballot(live);
  const uint64_t same_m = __ballot(live && q == q0);
  return live_m == same_m && (live_m & 1ull);
}

__device__ __forceinline__ uint32_t pack_cell(int x, int y, int z) {
  return (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20);
}

// Linear index of a cell: the (x, y) plane is cut into 4 x 4 tiles of z-rows; tiles are
// row-major, the 16 rows of a tile follow each other, z is fastest. Cells adjacent in z
// are adjacent in the index (a neighbour pencil z-1..z+1 is one run of buckets), and the
// rows that a tile's elements visit as neighbours mostly lie in the same tile, so they
// are read while still in L2.
__device__ __forceinline__ uint32_t cell_index(int nc, int x, int y, int z) {
  const int nt = (nc + 3) >> 2;
  return (uint32_t)(((((x >> 2) * nt + (y >> 2)) << 4) + (((x & 3) << 2) | (y & 3))) * nc + z);
}
__host__ __device__ __forceinline__ uint64_t cell_count(int nc) {
  const uint64_t nt = (uint64_t)((nc + 3) >> 2);
  return nt * nt * 16 * (uint64_t)nc;
}

// Bucket of a cell: its index modulo the (power-of-two) bucket count; when the grid has
// no more cells than buckets every cell has a bucket of its own.
__device__ __forceinline__ uint32_t bucket_of(int nc, uint32_t bmask, int x, int y, int z) {
  return cell_index(nc, x, y, z) & bmask;
}

// Exclusive scan of the tile totals into LDS: s_toff[t] = first sorted position of
// tile t, s_toff[ntiles] = number of hashed elements. Called by every thread.
__device__ __forceinline__ void block_tile_offsets(const int32_t* __restrict__ tile_tot,
                                                   int ntiles, int32_t* s_toff, int32_t* s_tmp) {
  const int t = threadIdx.x;
  const int nth = blockDim.x;
  const int per = (ntiles + nth - 1) / nth;
  const int beg = t * per;
  int sum = 0;
  for (int i = 0; i < per; ++i)
    if (beg + i < ntiles) sum += tile_tot[beg + i];
  s_tmp[t] = sum;
  __syncthreads();
  for (int o = 1; o < nth; o <<= 1) {
    const int add = t >= o ? s_tmp[t - o] : 0;
    __syncthreads();
    s_tmp[t] += add;
    __syncthreads();
  }
  int run = s_tmp[t] - sum;
  for (int i = 0; i < per; ++i)
    if (beg + i < ntiles) {
      s_toff[beg + i] = run;
      run += tile_tot[beg + i];
    }
  if (t == nth - 1) s_toff[ntiles] = s_tmp[nth - 1];
  __syncthreads();
}

// Grid for elements no larger than `ext`: the finest grid of cubic cells of edge >= ext
// that tiles the box (3 <= nc <= 1023); nc = 0 (no grid) when fewer than 3 fit.
__host__ __device__ inline Cells choose_cells(double box, double ext, double tol) {
  Cells c{};
  double h = ext > box / 1023.0 ? ext : box / 1023.0;
  int nc = (int)floor(box / h);
  if (nc > 1023) nc = 1023;
  if (nc < 3) nc = 0;
  c.nc = nc;
  c.fixed = 0;
  c.h = nc ? box / nc : box;
  c.inv_h = 1.0 / c.h;
  c.hlim = c.h - 4.0 * tol;
  c.h32 = (float)c.h;
  c.marg32 = (float)(c.h * 0x1p-16);
  return c;
}

// ---------------------------------------------------------------------------------
// step kernels
// ---------------------------------------------------------------------------------

// SCR: 0 = evolution only, 1 = FP64 screen data, 2 = FP32 screen data.
// Record of a point that stops at slice s (x = X[s][k], x_prev = X[s-1][k]); with_r
// adds the right neighbour's vertices X[s][j], X[s-1][j] (its next diamond's inputs).
__device__ __forceinline__ void write_frozen(semipar_point_rec* __restrict__ frz, const Slices& X,
                                             int ic, int ip, int k, int j, bool with_r, int face,
                                             int s, const int32_t* __restrict__ prv,
                                             const int64_t* __restrict__ id) {
  semipar_point_rec r;
  r.id = id[k];
  r.next_id = j >= 0 ? id[j] : -1;
  const int pk = prv[k];
  r.prev_id = pk >= 0 ? id[pk] : -1;
  r.step = s;
  r.flags = SEMIPAR_FLAG_FROZEN | (with_r ? SEMIPAR_FLAG_HAS_R : 0) | ((face + 1) << 8);
  const V4 a = ld(X, ic, k), b = ld(X, ip, k);
  r.x[0] = a.x; r.x[1] = a.y; r.x[2] = a.z; r.x[3] = a.t;
  r.x_prev[0] = b.x; r.x_prev[1] = b.y; r.x_prev[2] = b.z; r.x_prev[3] = b.t;
  if (with_r) {
    const V4 c = ld(X, ic, j), d = ld(X, ip, j);
    r.r[0] = c.x; r.r[1] = c.y; r.r[2] = c.z; r.r[3] = c.t;
    r.r_prev[0] = d.x; r.r_prev[1] = d.y; r.r_prev[2] = d.z; r.r_prev[3] = d.t;
  } else {
    for (int i = 0; i < 4; ++i) {
      r.r[i] = 0.0;
      r.r_prev[i] = 0.0;
    }
  }
  frz[k] = r;
}

// Runs of neighbouring lanes of a wave with the same bucket (lanes without one break
// runs). head: this lane starts a run of `len` lanes; first: the lane starting the run
// this lane is in. The lanes of a run share one atomic on their bucket's counter.
struct LaneRun {
  bool head;
  int len, first;
};
__device__ __forceinline__ LaneRun lane_run(bool has, uint32_t b) {
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t pb = __shfl_up(b, 1, 64);
  const bool ph = __shfl_up(has ? 1 : 0, 1, 64) != 0;
  LaneRun r;
  r.head = has && (lane == 0 || !ph || pb != b);
  const uint64_t heads = __ballot(r.head);
  const uint64_t inmask = __ballot(has);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0..lane
  const uint64_t after = (heads | ~inmask) & ~upto;  // run boundaries past this lane
  r.len = (after ? __ffsll((unsigned long long)after) - 1 : 64) - lane;
  const uint64_t hs = heads & upto;
  r.first = hs ? 63 - __clzll((long long)hs) : 0;
  return r;
}

// One step for every point: the diamond top X[n+1][k] (flat or first-order FRW) and,
// when SCR != 0, the element of band n (k to next[k]): FP64 box, cell, bucket count.
// BND: bounded region. Point k advances only when it is active, next[k] exists and is
// not stopped before this step, and the bottom X[n-1][next k] of its diamond lies in the
// region; otherwise it stops now (its record is written to frz). Its element exists when
// both k and next[k] advance; thread k re-derives next[k]'s decision from the same
// inputs. All decisions read the state before the step (a stop written in this step
// never satisfies "stopped before this step").
// HIST (a hand-off batch of a tiling run): inputs come from the world sheet by volume
// slot. Point k waits until its start step, then builds its diamond while the bottom
// X[n-1][next k] lies in its region (the same test every step, also at its start, where
// the token guarantees it) and stops for good at the first step where it does not. Each
// new vertex goes to the world sheet and, with the slice it stands on, to this batch's
// rings (for the elements); when it lies in another region than the point's previous
// vertex, that region's diamond of the left neighbour built on it gets a start token.
template <bool FRW, int SCR, bool BND, bool HIST = false>
__global__ __launch_bounds__(NT) void k_evolve(Slices X, const int32_t* __restrict__ nxt,
                                               const int32_t* __restrict__ prv,
                                               const int64_t* __restrict__ id, int n,
                                               sp::Period P, double hcoef, Ctrl* ctrl, HashCfg hc,
                                               void* __restrict__ ebox,
                                               int32_t* __restrict__ ecell,
                                               int32_t* __restrict__ cnt,
                                               LargeBox* __restrict__ large,
                                               uint64_t* __restrict__ blkred,
                                               int32_t* __restrict__ fstep,
                                               int32_t* __restrict__ face,
                                               semipar_point_rec* __restrict__ frz, RegionGeom G0,
                                               const RegionGeom* __restrict__ geoms,
                                               const int32_t* __restrict__ rid,
                                               const RCell* __restrict__ rcell,
                                               uint64_t* __restrict__ rext,
                                               uint8_t* __restrict__ wlive, HistCfg hs,
                                               const int32_t* __restrict__ act) {
  if (ctrl->done) return;
  const int s = ctrl->step;
  const Cells cs = ctrl->cells;
  const int nw = (n + 63) >> 6;
  const int ic = s % 3, ip = (s + 2) % 3, in = (s + 1) % 3;
  // grid-stride over the points in slot order (neighbouring lanes read neighbouring
  // slots, so the SoA loads stay coalesced), with the same trip count for every thread
  // so that wave-wide operations stay uniform; a bounded region walks its list of the
  // points that still advanced at the start of this block of steps (ascending slots)
  const bool list = act != nullptr;
  const int nn = list ? ctrl->n_act : n;
  const int span = gridDim.x * NT;
  const int iters = (nn + span - 1) / span;
  uint64_t tkey = KEY_MAX;
  uint64_t xkey = 0;
  uint32_t nadv = 0;
  for (int it = 0; it < iters; ++it) {
  const int ii = it * span + blockIdx.x * NT + threadIdx.x;
  // a wave of 64 slots none of which still advances is skipped: its flag was cleared by
  // the step that stopped its last point, and stopped points never advance again
  const int wv = __builtin_amdgcn_readfirstlane(ii >> 6);
  if (!list && wv < nw && !wlive[wv]) continue;
  if (list && ii - (ii & 63) >= nn) continue;  // (a whole wave past the list's end)
  const int k = ii < nn ? (list ? act[ii] : ii) : n;
  uint64_t xk = 0;  // this point's element extent
  bool still = false;  // k advanced in this step (and so is still active)
  bool hashed = false;  // k's element goes to bucket hbk of the spatial hash
  uint32_t hbk = 0;
  // a point of a bounded region that stopped before this step, or a point of a removed
  // loop (fstep is then passed for a whole-volume region too), has nothing to do (its
  // element cell already reads NO_ELEM)
  bool live_pt = k < n;
  if constexpr (BND) live_pt = live_pt && fstep[k] == FS_ACTIVE;
  else live_pt = live_pt && (!fstep || fstep[k] == FS_ACTIVE);
  V4 L, R, B;
  int64_t my_name = 0;
  int g = 0, gj = 0;
  if (live_pt) {
    bool adv = true;
    int j = nxt[k];
    // geometry of k's region (links never leave a region, so also next[k]'s)
    RegionGeom G;
    if constexpr (BND) G = rid ? geoms[rid[k]] : G0;
    if constexpr (HIST) {
      adv = false;
      const int32_t s_start = hs.start[k];
      if (s < s_start) {
        still = true;  // not started yet: its wave stays live
      } else if (s - hs.s0 >= hs.ns) {
        atomicOr(&ctrl->err, HERR_SLICES);  // (nothing on slice s was ever written)
        fstep[k] = s;
      } else {
        g = hs.gsl[k];
        gj = hs.gnx[k];
        my_name = hs.sname[rid[k]];
        if (ldhome(hs, s - 1, gj) == my_name) {
          B = ldh(hs, s - 1, gj);
          L = ldh(hs, s, g);
          R = ldh(hs, s, gj);
          if (!(B.t == B.t && L.t == L.t && R.t == R.t)) {
            atomicOr(&ctrl->err, HERR_INPUT);
            fstep[k] = s;
          } else {
            adv = true;
          }
        } else {
          if (s == s_start) atomicOr(&ctrl->err, HERR_START);
          fstep[k] = s;
        }
      }
    } else if constexpr (BND) {
      adv = false;
      {
        int f = -1;
        bool with_r = false;
        if (j < 0) {
          f = -1;
        } else if (fstep[j] < s) {
          f = face[j];
        } else {
          f = exit_face(G, ld(X, ip, j));
          if (f < 0) adv = true;
          with_r = true;
        }
        if (!adv) {
          write_frozen(frz, X, ic, ip, k, j, with_r, f, s, prv, id);
          face[k] = f;
          fstep[k] = s;
        }
      }
    }
    if (adv) {
      nadv += 1;
      still = true;
      if constexpr (!HIST) {
        L = ld(X, ic, k);
        R = ld(X, ic, j);
        B = ld(X, ip, j);
      }
      const V4 T = sp::top<FRW>(L, R, B, P, hcoef);
      st(X, in, k, T);
      if constexpr (HIST) {
        st(X, ic, k, L);
        // T's home, from the homes of L, R and B (B's is this region's)
        const int64_t hl = ldhome(hs, s, g);
        bool tie = false;
        const int64_t tn = resolve_home(hist_name(hs, T), hl, ldhome(hs, s, gj), my_name, &tie);
        if (tie) atomicOr(&ctrl->err, HERR_TIE);
        if (s + 1 - hs.s0 < hs.ns) {
          const int64_t at = (int64_t)(s + 1 - hs.s0) * hs.n + g;
          hs.H[at] = make_double4(T.x, T.y, T.z, T.t);
          hs.home[at] = tn;
        } else {
          atomicOr(&ctrl->err, HERR_SLICES);
        }
        // the diamond of k's left neighbour with bottom T belongs to T's home; its start
        // there is announced when T is the first vertex of k's world line homed there
        if (tn != hl) {
          if (tn == my_name) {
            atomicOr(&ctrl->err, HERR_SELF);
          } else {
            const int32_t dest = hist_region(hs, tn);
            if (dest >= 0) {
              const unsigned long long w =
                  atomicAdd((unsigned long long*)&ctrl->tok_n, 1ull);
              if ((int64_t)w < hs.tok_cap) {
                HandTok tkn;
                tkn.slot = hs.gprev[g];
                tkn.step = s + 2;
                tkn.region = dest;
                tkn.pad = 0;
                hs.tok[w] = tkn;
              } else {
                atomicOr(&ctrl->err, HERR_TOKENS);
              }
            }
          }
        }
      }
      const uint64_t tk = order_key(T.t);
      tkey = tk < tkey ? tk : tkey;
      if constexpr (SCR != 0) {
        const int jj = HIST ? -1 : nxt[j];  // (a hand-off batch reads next[j] by volume slot)
        bool jadv = true;
        V4 Rj, Bj;
        if constexpr (HIST) {
          // next[k] builds its diamond in this region at this step: it is here, has
          // started, has not stopped before, and its own bottom lies in the region
          jadv = j >= 0 && hs.start[j] <= s && fstep[j] >= s;
          if (jadv) {
            const int gjj = hs.gnx[j];
            jadv = ldhome(hs, s - 1, gjj) == my_name;
            if (jadv) {
              Bj = ldh(hs, s - 1, gjj);
              Rj = ldh(hs, s, gjj);
              jadv = Bj.t == Bj.t && Rj.t == Rj.t;
            }
          }
        } else if constexpr (BND) {
          jadv = fstep[j] == FS_ACTIVE && jj >= 0 && fstep[jj] >= s;
          if (jadv) {
            Bj = ld(X, ip, jj);
            jadv = exit_face(G, Bj) < 0;
          }
          if (jadv) Rj = ld(X, ic, jj);
        } else {
          Rj = ld(X, ic, jj);
          Bj = ld(X, ip, jj);
        }
        if (!jadv) {
          ecell[k] = NO_ELEM;
        } else {
          const V4 Tj = sp::top<FRW>(R, Rj, Bj, P, hcoef);
          const Elem e = sp::make_elem(L, R, T, Tj, P);
          const Box4 b = sp::elem_box(e);
          double ext = b.hi[0] - b.lo[0];
          ext = fmax(ext, b.hi[1] - b.lo[1]);
          ext = fmax(ext, b.hi[2] - b.lo[2]);
          xk = order_key(ext);
          double W[3], w[3];
          for (int c = 0; c < 3; ++c) {
            W[c] = P.box * floor(b.lo[c] * P.inv);
            w[c] = b.lo[c] - W[c];
          }
          const bool local = BND && rcell != nullptr;
          RCell C{};
          if (local) C = rcell[rid[k]];
          if (local ? !(ext <= C.hlim) : (cs.nc == 0 || !(ext <= cs.hlim))) {
            const int li = atomicAdd(&ctrl->n_large, 1);
            LargeBox lb;
            for (int c = 0; c < 3; ++c) {
              lb.wl[c] = w[c];
              lb.ext[c] = b.hi[c] - b.lo[c];
            }
            lb.tlo = b.lo[3];
            lb.thi = b.hi[3];
            lb.slot = k;
            lb.pad = 0;
            large[li] = lb;
            ecell[k] = -1 - li;
          } else {
            int ci[3];
            double lor[3], hir[3];
            if (local) {
              // coordinates relative to the region's grid origin, in the periodic image
              // nearest the grid's centre (a box of only twice the region's reach puts
              // the far side of the grid more than half a box from its origin)
              const double o[3] = {C.ox, C.oy, C.oz};
              const double half = 0.5 * (double)C.nc * C.h;
              for (int c = 0; c < 3; ++c) {
                const double d = b.lo[c] - o[c];
                const double sh = P.box * P.nearest(d - half);
                const double dl = d - sh;
                int q = (int)floor(dl * C.inv_h);
                q = q < 0 ? 0 : (q > C.nc - 1 ? C.nc - 1 : q);
                ci[c] = q;
                lor[c] = dl - (double)q * C.h;
                hir[c] = ((b.hi[c] - o[c]) - sh) - (double)q * C.h;
              }
            } else {
              for (int c = 0; c < 3; ++c) {
                int q = (int)floor(w[c] * cs.inv_h);
                q = q < 0 ? 0 : (q > cs.nc - 1 ? cs.nc - 1 : q);
                ci[c] = q;
                lor[c] = w[c] - (double)q * cs.h;
                hir[c] = (b.hi[c] - W[c]) - (double)q * cs.h;
              }
            }
            if constexpr (SCR == 1) {
              double4* o = (double4*)ebox + (size_t)k * 2;
              o[0] = make_double4(lor[0], lor[1], lor[2], b.lo[3]);
              o[1] = make_double4(hir[0], hir[1], hir[2], b.hi[3]);
            } else {
              float4* o = (float4*)ebox + (size_t)k * 2;
              o[0] = make_float4(__double2float_rd(lor[0] - hc.tol),
                                 __double2float_rd(lor[1] - hc.tol),
                                 __double2float_rd(lor[2] - hc.tol),
                                 __double2float_rd((b.lo[3] - hc.tref) - hc.tol_t));
              o[1] = make_float4(__double2float_ru(hir[0] + hc.tol),
                                 __double2float_ru(hir[1] + hc.tol),
                                 __double2float_ru(hir[2] + hc.tol),
                                 __double2float_ru((b.hi[3] - hc.tref) + hc.tol_t));
            }
            const uint32_t bk =
                local ? (C.base + cell_index(C.nc, ci[0], ci[1], ci[2])) & hc.bmask
                      : bucket_of(cs.nc, hc.bmask, ci[0], ci[1], ci[2]);
            hashed = true;
            hbk = bk;
            ecell[k] = (int32_t)pack_cell(ci[0], ci[1], ci[2]);
          }
        }
      }
    } else if constexpr (SCR != 0) {
      ecell[k] = NO_ELEM;
    }
  }
  // bucket counts: neighbouring lanes are neighbouring points of a string and often share
  // a cell, so each run of lanes with one bucket adds its size with a single atomic,
  // whose result nobody waits for (k_scatter takes the places)
  if constexpr (SCR != 0) {
    const LaneRun lr = lane_run(hashed, hbk);
    if (lr.head) atomicAdd(&cnt[hbk], lr.len);
  }
  // batch: largest element extent per sub-region (one atomic per wave when the wave
  // holds one sub-region)
  if constexpr (BND && SCR != 0) {
    if (rext) {
      const bool live = k < n;
      const int q = live ? rid[k] : -1;
      const int q0 = __shfl(q, 0, 64);
      const uint64_t lm = __ballot(live), sm = __ballot(live && q == q0);
      if (lm == sm && (lm & 1ull)) {
        const uint64_t m = wave_max_u64(xk);
        if ((threadIdx.x & 63) == 0 && m != 0)
          atomicMax((unsigned long long*)&rext[(size_t)q0 * REXT_STRIDE], m);
      } else if (live && xk != 0) {
        atomicMax((unsigned long long*)&rext[(size_t)q * REXT_STRIDE], xk);
      }
    }
  }
  xkey = xk > xkey ? xk : xkey;
  if (!list) {
    const uint64_t any = __ballot(still);
    if ((threadIdx.x & 63) == 0 && wv < nw) wlive[wv] = any != 0ull ? 1 : 0;
  }
  }  // grid-stride loop
  // per block: minimum t of the new slice, largest element extent, points advanced;
  // reduced by k_resolve (no same-address atomics across the grid)
  __shared__ uint64_t wmin[NT / 64], wmax[NT / 64];
  __shared__ uint32_t wadv[NT / 64];
  tkey = wave_min_u64(tkey);
  xkey = wave_max_u64(xkey);
  for (int o = 32; o > 0; o >>= 1) nadv += __shfl_xor(nadv, o, 64);
  if ((threadIdx.x & 63) == 0) {
    wmin[threadIdx.x >> 6] = tkey;
    wmax[threadIdx.x >> 6] = xkey;
    wadv[threadIdx.x >> 6] = nadv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t m = wmin[0], x = wmax[0];
    uint64_t a = wadv[0];
    for (int w = 1; w < NT / 64; ++w) {
      m = wmin[w] < m ? wmin[w] : m;
      x = wmax[w] > x ? wmax[w] : x;
      a += wadv[w];
    }
    blkred[4 * blockIdx.x] = m;
    blkred[4 * blockIdx.x + 1] = x;
    blkred[4 * blockIdx.x + 2] = a;
  }
}

constexpr int MAX_TILES = 2048;  // buckets <= 2^23

// Per-tile exclusive scan of the bucket counts (k_scatter takes them back to zero);
// tile totals go to tile_tot, which k_toff scans. (The last workgroup could scan them
// instead, but making the totals visible to it takes a device-scope fence in every
// workgroup, which writes back the L2: 12 times slower than a second launch.)
__global__ __launch_bounds__(256) void k_scan(int32_t* __restrict__ cnt, int32_t* __restrict__ loc,
                                              int32_t* __restrict__ tile_tot, const Ctrl* ctrl) {
  if (ctrl->done) return;
  __shared__ int32_t sh[256];
  const int t = threadIdx.x;
  const size_t base = (size_t)blockIdx.x * TS + (size_t)t * 16;
  int4* c4 = (int4*)(cnt + base);
  int v[16];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int4 q = c4[i];
    v[4 * i] = q.x;
    v[4 * i + 1] = q.y;
    v[4 * i + 2] = q.z;
    v[4 * i + 3] = q.w;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) sum += v[i];
  sh[t] = sum;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int add = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int run = sh[t] - sum;
  int out[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    out[i] = run;
    run += v[i];
  }
  int4* l4 = (int4*)(loc + base);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    l4[i] = make_int4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
  }
  if (t == 255) tile_tot[blockIdx.x] = sh[255];
}

constexpr int POINT_GRID = 2048;  // most workgroups of the grid-stride per-point kernels

constexpr int SCREEN_GRID = 2560;  // most workgroups of the screen (a multiple of 8)
constexpr int LARGE_GRID = 256;    // workgroups of k_screen_large (a wave per large element)
constexpr int LARGE_CELLS = 4096;  // most cells a large element's wave visits one by one

__device__ __forceinline__ int bucket_start(const int32_t* loc, const int32_t* s_toff, uint32_t b) {
  return loc[b] + s_toff[b >> TS_LOG];
}

// Exclusive scan of the tile totals (one workgroup): toff[t] = first sorted position of
// tile t, toff[ntiles] = number of hashed elements.
__global__ __launch_bounds__(1024) void k_toff(const int32_t* __restrict__ tile_tot, int ntiles,
                                               int32_t* __restrict__ toff, const Ctrl* ctrl) {
  if (ctrl->done) return;
  __shared__ int32_t s_toff[MAX_TILES + 1];
  __shared__ int32_t s_tmp[1024];
  block_tile_offsets(tile_tot, ntiles, s_toff, s_tmp);
  for (int i = threadIdx.x; i <= ntiles; i += 1024) toff[i] = s_toff[i];
}

// Neighbour pencils of a sorted element (64 bytes), written by k_scatter for the screen
// variant that reads them instead of looking them up (k_screen_pre). Pencil 0 is the
// element's own z-row from its own cell: [pos + 1, re0). Pencils 1..4 are the rows
// (x, y+1), (x+1, y-1), (x+1, y), (x+1, y+1), cells z-1 .. z+1: [rb, re). msk bits
// 3p .. 3p+2 say which of the cells z-1, z, z+1 of pencil p exist; bit 15 + p says that
// pencil p's cells are not consecutive buckets (the screen then looks them up one by
// one). nk, pk are the slots of the element's point's neighbours, salt the key salt and
// h32, marg32 the cell edge and FP32 slack of its grid.
constexpr int N_PENCIL = 5;  // forward half shell of a cell: 5 z-pencils of 3 cells
struct PencilAux {
  int32_t re0;
  int32_t rb[4], re[4];
  uint32_t msk;
  int32_t nk, pk;
  uint32_t salt;
  float h32, marg32;
  int32_t pad;
};
static_assert(sizeof(PencilAux) == 64, "four 16-byte loads");

__device__ __forceinline__ void pencil_offsets(int p, int& dx, int& dy) {
  dx = p == 0 ? 0 : (p == 1 ? 0 : 1);
  dy = p == 0 ? 0 : (p == 1 ? 1 : p - 3);
}

// Cell-sorted copies of each hashed element: cell key, slot and screen box. In a batch
// the key is the packed local cell xor the sub-region's salt.
template <int SCR>
__global__ __launch_bounds__(NT) void k_scatter(int n, const int32_t* __restrict__ ecell,
                                                int32_t* __restrict__ cnt,
                                                const int32_t* __restrict__ loc,
                                                const int32_t* __restrict__ toff,
                                                const void* __restrict__ ebox,
                                                int2* __restrict__ sent,
                                                void* __restrict__ sbox, HashCfg hc,
                                                const int32_t* __restrict__ rid,
                                                const RCell* __restrict__ rcell,
                                                const uint8_t* __restrict__ wlive,
                                                const Ctrl* ctrl,
                                                PencilAux* __restrict__ saux,
                                                const int32_t* __restrict__ nxt,
                                                const int32_t* __restrict__ prv,
                                                const int32_t* __restrict__ act) {
  if (ctrl->done) return;
  const int nc = ctrl->cells.nc;
  const Cells cs = ctrl->cells;
  const int nw = (n + 63) >> 6;
  // the same trip count for every thread (wave-wide run detection below); a bounded
  // region walks its list of advancing points, which holds every element of the step
  const bool list = act != nullptr;
  const int nn = list ? ctrl->n_act : n;
  const int span = gridDim.x * NT;
  const int iters = (nn + span - 1) / span;
  for (int it = 0; it < iters; ++it) {
  const int ii = it * span + blockIdx.x * NT + threadIdx.x;
  // no point of a cleared wave advanced this step, so none has an element
  const int wv = __builtin_amdgcn_readfirstlane(ii >> 6);
  if (!list && (wv >= nw || !wlive[wv])) continue;
  if (list && ii - (ii & 63) >= nn) continue;  // (a whole wave past the list's end)
  const int k = ii < nn ? (list ? act[ii] : ii) : n;
  const int32_t c = k < n ? ecell[k] : -1;
  const bool has = c >= 0;
  const int x = c & 1023, y = (c >> 10) & 1023, z = (c >> 20) & 1023;
  uint32_t b = 0;
  int32_t key = c;
  RCell C{};
  if (has) {
    if (rcell) {
      C = rcell[rid[k]];
      b = (C.base + cell_index(C.nc, x, y, z)) & hc.bmask;
      key = (int32_t)((uint32_t)c ^ C.salt);
    } else {
      b = bucket_of(nc, hc.bmask, x, y, z);
    }
  }
  // places in the bucket: each run of lanes with one bucket takes the top places left
  // by one atomic decrement of its count (which so returns to zero for the next step)
  const LaneRun lr = lane_run(has, b);
  int base = 0;
  if (lr.head) base = atomicSub(&cnt[b], lr.len) - lr.len;
  base = __shfl(base, lr.first, 64) + ((int)(threadIdx.x & 63) - lr.first);
  if (!has) continue;
  const int pos = bucket_start(loc, toff, b) + base;
  if (saux) {
    // the five neighbour pencils' ranges of sorted entries (the screen's lookups, done
    // here where the element's grid and bucket offsets are already at hand)
    const bool local = rcell != nullptr;
    const int gnc = local ? C.nc : nc;
    auto bucket = [&](int xx, int yy, int zz) -> uint32_t {
      return local ? (C.base + cell_index(gnc, xx, yy, zz)) & hc.bmask
                   : bucket_of(gnc, hc.bmask, xx, yy, zz);
    };
    auto wrapc = [&](int v) { return v < 0 ? v + gnc : (v >= gnc ? v - gnc : v); };
    PencilAux A{};
    A.nk = nxt[k];
    A.pk = prv[k];
    A.salt = local ? C.salt : 0u;
    A.h32 = local ? C.h32 : cs.h32;
    A.marg32 = local ? C.marg32 : cs.marg32;
    uint32_t msk = 0;
#pragma unroll
    for (int p = 0; p < N_PENCIL; ++p) {
      int dx, dy;
      pencil_offsets(p, dx, dy);
      int xx = x + dx, yy = y + dy;
      if (local) {
        if (xx >= gnc || yy < 0 || yy >= gnc) continue;  // no such row: no cells
      } else {
        xx = wrapc(xx);
        yy = wrapc(yy);
      }
      bool kv[3];
      uint32_t bk[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int dz = u - 1;
        int zz = z + dz;
        bool v = !(p == 0 && dz < 0);
        if (local) v = v && zz >= 0 && zz < gnc;
        else zz = wrapc(zz);
        kv[u] = v;
        bk[u] = bucket(xx, yy, zz);
      }
      const int first = kv[0] ? 0 : 1;
      const int last = kv[2] ? 2 : 1;
      bool consec = true;
      if (first == 0) consec = consec && bk[1] == bk[0] + 1;
      if (last == 2) consec = consec && bk[2] == bk[1] + 1;
      msk |= (uint32_t)((kv[0] ? 1 : 0) | 2 | (kv[2] ? 4 : 0)) << (3 * p);
      if (!consec) {
        msk |= 1u << (15 + p);
        continue;
      }
      const int end = bucket_start(loc, toff, (last == 2 ? bk[2] : bk[1]) + 1);
      if (p == 0) {
        A.re0 = end;
      } else {
        A.rb[p - 1] = bucket_start(loc, toff, first == 0 ? bk[0] : bk[1]);
        A.re[p - 1] = end;
      }
    }
    A.msk = msk;
    saux[pos] = A;
  }
  if constexpr (SCR == 1) {
    sent[pos] = make_int2(key, k);
    const double4* src = (const double4*)ebox + (size_t)k * 2;
    double4* dst = (double4*)sbox + (size_t)pos * 2;
    dst[0] = src[0];
    dst[1] = src[1];
  } else {
    // (lo.xyz, key), (hi.xyz, slot): the screen's spatial box with its key and slot
    const float4* src = (const float4*)ebox + (size_t)k * 2;
    float4* dst = (float4*)sbox + (size_t)pos * 2;
    float4 lo = src[0], hi = src[1];
    lo.w = __int_as_float(key);
    hi.w = __int_as_float(k);
    dst[0] = lo;
    dst[1] = hi;
  }
  }  // grid-stride loop
}

__device__ __forceinline__ void push_cand(Ctrl* ctrl, int2* cand, int cap, int k, int m) {
  const int i = atomicAdd(&ctrl->n_cand, 1);
  if (i < cap) cand[i] = make_int2(k, m);
}

// Periodic 1-D overlap of [a, a + ea] and [b, b + eb] on a circle of length box.
__device__ __forceinline__ bool wrap_overlap(double a, double ea, double b, double eb,
                                             const sp::Period& P, double tol) {
  const double box = P.box;
  double d = b - a;
  d = d - box * floor(d * P.inv);
  return d <= ea + tol || (box - d) <= eb + tol;
}

// Screen box of a sorted entry (lo xyz t, hi xyz t), loaded as two 16/32-byte vectors.
template <class T>
struct SBox {
  T v[8];
};
template <class T>
__device__ __forceinline__ SBox<T> load_sbox(const void* sbox, int q) {
  SBox<T> b;
  if constexpr (sizeof(T) == 8) {
    const double4* p = (const double4*)sbox + (size_t)q * 2;
    const double4 a = p[0], c = p[1];
    b.v[0] = a.x; b.v[1] = a.y; b.v[2] = a.z; b.v[3] = a.w;
    b.v[4] = c.x; b.v[5] = c.y; b.v[6] = c.z; b.v[7] = c.w;
  } else {
    const float4* p = (const float4*)sbox + (size_t)q * 2;
    const float4 a = p[0], c = p[1];
    b.v[0] = a.x; b.v[1] = a.y; b.v[2] = a.z; b.v[3] = a.w;
    b.v[4] = c.x; b.v[5] = c.y; b.v[6] = c.z; b.v[7] = c.w;
  }
  return b;
}

// Spatial overlap of box a with box b shifted by (sx, sy, sz), slack tl. The screen
// tests space only: the time ranges of elements of one band that are close in space
// nearly always overlap, and the FP64 confirmation tests the exact 4-D boxes, so leaving
// time out only admits a few more candidates (in either precision).
template <class T>
__device__ __forceinline__ bool box_overlap(const SBox<T>& a, const SBox<T>& b, T sx, T sy, T sz,
                                            T tl) {
  return a.v[0] <= b.v[4] + sx + tl && b.v[0] + sx <= a.v[4] + tl && a.v[1] <= b.v[5] + sy + tl &&
         b.v[1] + sy <= a.v[5] + tl && a.v[2] <= b.v[6] + sz + tl && b.v[2] + sz <= a.v[6] + tl;
}

// Which of the cells one step up an axis (+x, +y, +z) box a can reach. Such a cell holds
// entries whose low corner is at least one cell edge hh above a's cell origin, less the
// rounding of that corner (a few times the tolerance tol): when a's high side plus the
// slack tl stays below the edge less a margin (1/256 of it plus eight tolerances, far
// above every rounding of these sums), box_overlap fails for all of them.
template <class T>
__device__ __forceinline__ void reach_up(const SBox<T>& a, T hh, T tl, double tol, bool (&up)[3]) {
  const T gate = hh - (hh * (T)0x1p-8 + (T)(8.0 * tol));
#pragma unroll
  for (int i = 0; i < 3; ++i) up[i] = a.v[4 + i] + tl >= gate;
}

// The FP32 screen's sorted entries carry their cell key and slot in the fourth component
// of the two float4 (lo.xyz, key) and (hi.xyz, slot), where the time range would be: one
// 32-byte entry per element, read with two loads.
template <int SCR>
__device__ __forceinline__ int2 entry_key_slot(const int2* __restrict__ sent,
                                               const SBox<typename std::conditional<SCR == 1, double, float>::type>& b,
                                               int q) {
  if constexpr (SCR == 2) return make_int2(__float_as_int(b.v[3]), __float_as_int(b.v[7]));
  else return sent[q];
}

// Key and slot of sorted entry q (FP32: from the box's fourth components).
template <int SCR>
__device__ __forceinline__ int2 sent_key_slot(const int2* __restrict__ sent, const void* sbox,
                                              int q) {
  if constexpr (SCR == 2) {
    const float4* p = (const float4*)sbox + (size_t)q * 2;
    return make_int2(__float_as_int(p[0].w), __float_as_int(p[1].w));
  } else {
    return sent[q];
  }
}

constexpr int SBUF = 1024;       // candidates staged in LDS per block (more go straight to memory)
constexpr int SBUF_FLUSH = 512;  // staged candidates are written out from this many on

// Workgroups are handed to the 8 XCDs of the chip in turn (workgroup i to XCD i mod 8),
// each XCD with its own L2. xcd_block() renumbers a 1-D grid of 8*ceil(total/8)
// workgroups so that XCD x runs the logical blocks [x*per, (x+1)*per): consecutive logical
// blocks then share one L2. Returns a value >= total for the padding workgroups.
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_block(int total) {
  const int lin = blockIdx.x;
  const int per = (total + N_XCD - 1) / N_XCD;
  return (lin % N_XCD) * per + lin / N_XCD;
}
inline int xcd_grid(int total) { return (total + N_XCD - 1) / N_XCD * N_XCD; }

// Half-shell screen over the cell-sorted elements, by z-pencils. The element at sorted
// position q (cell (x, y, z)) is tested against
//   pencil 0: the later entries of its own cell and every entry of cell (x, y, z+1);
//   pencils 1..4: every entry of the cells (x', y', z-1 .. z+1) for
//                 (x', y') = (x, y+1), (x+1, y-1), (x+1, y), (x+1, y+1),
// i.e. the 14 cells of the forward half shell. Buckets are row-major in the cell index
// with z fastest, so a pencil's cells are consecutive buckets and one range of the
// sorted entries: 5 range lookups per element instead of 14. Where a pencil's buckets
// are not consecutive (periodic wrap in z, end of the bucket table) its cells are
// looked up one by one. Entries of other cells sharing a bucket are skipped by key.
// G threads share an element (G = 1: all pencils; G = 5: one pencil each); thread
// g = 0 also tests the element against every large element (two large ones: by the
// one of smaller slot). Threads past the hashed elements take one large element each.
// Each unordered pair is tested exactly once. Logical block = (element block, g),
// renumbered per XCD (xcd_block).
constexpr int SCREEN_EPW = 12;  // elements per wave when five lanes share an element
constexpr int SPLIT_PRE = 2;    // screen variant: pencils precomputed by k_scatter

template <int SCR, int G>
__global__ __launch_bounds__(NT, (SCR == 2 && G == 1) ? 5 : 1) void k_screen(int n, const int2* __restrict__ sent,
                                               const void* __restrict__ sbox,
                                               const void* __restrict__ ebox_slot,
                                               const int32_t* __restrict__ nxt,
                                               const int32_t* __restrict__ prv,
                                               const int32_t* __restrict__ loc,
                                               const int32_t* __restrict__ toff, int ntiles,
                                               const LargeBox* __restrict__ large, HashCfg hc,
                                               sp::Period P, int2* __restrict__ cand, int cap,
                                               Ctrl* ctrl,
                                               const int32_t* __restrict__ rid,
                                               const RCell* __restrict__ rcell) {
  static_assert(G == 1 || G == N_PENCIL, "one or five threads per element");
  if (ctrl->done) return;
  using T = typename std::conditional<SCR == 1, double, float>::type;
  __shared__ int2 sbuf[SBUF];
  __shared__ int s_cnt, s_base;
  const Cells cs = ctrl->cells;
  const int nl = ctrl->n_large;
  const int n_norm = toff[ntiles];
  // The grid is sized for the resident workgroups, not for the points: the blocks of
  // each XCD walk a contiguous range of element chunks (neighbouring cells, shared L2)
  // and stop at this step's hashed + large element count, read on the device.
  constexpr int EPB = G == 1 ? NT : (NT / 64) * SCREEN_EPW;  // elements per chunk
  const int nchunk = (n_norm + nl + EPB - 1) / EPB;
  const int cper = (nchunk + N_XCD - 1) / N_XCD;
  const int xcd = (int)blockIdx.x % N_XCD;
  const int bper = (int)gridDim.x / N_XCD;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  for (int c = (int)blockIdx.x / N_XCD; c < cper; c += bper) {
  const int lid = xcd * cper + c;
  if (lid >= nchunk) break;
  // the block's last chunk: the staged candidates are written out after it
  const bool last = c + bper >= cper || lid + bper >= nchunk;
  // G = 1: one element per thread. G = 5: an element's five threads are neighbouring
  // lanes of one wave (12 elements per wave, lanes 60..63 idle), so their identical
  // loads of the element's own data are served by one request.
  int q, g;
  if constexpr (G == 1) {
    q = lid * NT + (int)threadIdx.x;
    g = 0;
  } else {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    g = lane % N_PENCIL;
    q = lane < SCREEN_EPW * N_PENCIL ? (lid * (NT / 64) + wv) * SCREEN_EPW + lane / N_PENCIL
                                      : INT_MAX;
  }
  auto push = [&](int a, int b) {
    const int i = atomicAdd(&s_cnt, 1);
    if (i < SBUF)
      sbuf[i] = make_int2(a, b);
    else
      push_cand(ctrl, cand, cap, a, b);
  };
  if (q < n_norm + nl && (q < n_norm || g == 0)) {
    int k;
    bool own_large;
    double wl[3], ex[3], tlo, thi;  // wrapped box of the element (for large partners)
    if (q < n_norm) {
      own_large = false;
      const SBox<T> me = load_sbox<T>(sbox, q);
      const int2 ent = entry_key_slot<SCR>(sent, me, q);
      k = ent.y;
      // grid of the element: the region's own (batch) or the periodic box's
      RCell C{};
      uint32_t salt = 0;
      int gnc = cs.nc;
      const bool local = rcell != nullptr;
      if (local) {
        C = rcell[rid[k]];
        salt = C.salt;
        gnc = C.nc;
      }
      const int32_t c = (int32_t)((uint32_t)ent.x ^ salt);
      const int nk = nxt[k], pk = prv[k];
      const int cx = c & 1023, cy = (c >> 10) & 1023, cz = (c >> 20) & 1023;
      const T tl = SCR == 1 ? (T)hc.tol : (T)(local ? C.marg32 : cs.marg32);
      const T hh = SCR == 1 ? (T)(local ? C.h : cs.h) : (T)(local ? C.h32 : cs.h32);
      auto bucket = [&](int x, int y, int z) -> uint32_t {
        return local ? (C.base + cell_index(gnc, x, y, z)) & hc.bmask
                     : bucket_of(gnc, hc.bmask, x, y, z);
      };
      auto wrapc = [&](int v) { return v < 0 ? v + gnc : (v >= gnc ? v - gnc : v); };
      // test the entries [beg, end) whose key is that of the pencil cell z + dz for a
      // dz in {-1, 0, 1} with valid bit set (kv[dz + 1])
      auto scan = [&](int beg, int end, const int32_t (&kk)[3], const bool (&kv)[3], int dx,
                      int dy) {
        const T sx = (T)dx * hh, sy = (T)dy * hh;
        auto test = [&](const int2 e, const SBox<T>& b) {
          int dz = 2;
#pragma unroll
          for (int u = 0; u < 3; ++u)
            if (kv[u] && e.x == kk[u]) dz = u - 1;
          const int m = e.y;
          if (dz != 2 && m != nk && m != pk && box_overlap(me, b, sx, sy, (T)dz * hh, tl))
            push(k, m);
        };
        int q2 = beg;
        // four entries at a time: independent loads in flight together
        for (; q2 + 4 <= end; q2 += 4) {
          int2 e4[4];
          SBox<T> b4[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            b4[v] = load_sbox<T>(sbox, q2 + v);
            e4[v] = entry_key_slot<SCR>(sent, b4[v], q2 + v);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) test(e4[v], b4[v]);
        }
        for (; q2 < end; ++q2) {
          const SBox<T> b1 = load_sbox<T>(sbox, q2);
          test(entry_key_slot<SCR>(sent, b1, q2), b1);
        }
      };
      // phase 1: every pencil's entry range (all bucket-offset loads issued before any
      // range is scanned). A pencil whose cells are consecutive buckets is kept as one
      // range, its centre cell key (unsalted) and a mask of its valid cells: cell z+dz
      // has key centre + dz * 2^20 (z lies in bits 20..29 and does not wrap then).
      // Pencils whose buckets are not consecutive are scanned cell by cell right here.
      constexpr int NPT = (N_PENCIL + G - 1) / G;  // pencils per thread
      int rb[NPT], re[NPT], cen[NPT], msk[NPT];
      bool up[3];  // cells one step up an axis that the element cannot reach are not read
      reach_up(me, hh, tl, hc.tol, up);
#pragma unroll
      for (int pi = 0; pi < NPT; ++pi) {
        const int p = g + pi * G;
        rb[pi] = 0;
        re[pi] = 0;
        cen[pi] = 0;
        msk[pi] = 0;
        if (p >= N_PENCIL) continue;
        const int dx = p == 0 ? 0 : (p == 1 ? 0 : 1);
        const int dy = p == 0 ? 0 : (p == 1 ? 1 : p - 3);
        if ((dx == 1 && !up[0]) || (dy == 1 && !up[1])) continue;
        int x = cx + dx, y = cy + dy;
        if (local) {
          if (x >= gnc || y < 0 || y >= gnc) continue;
        } else {
          x = wrapc(x);
          y = wrapc(y);
        }
        // the pencil's cells z + dz: dz = 0, 1 (pencil 0, own cell from q + 1) or -1, 0, 1
        bool kv[3];
        int32_t kk[3];
        uint32_t bk[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          const int dz = u - 1;
          int z = cz + dz;
          bool v = !(p == 0 && dz < 0) && (dz < 1 || up[2]);
          if (local) {
            v = v && z >= 0 && z < gnc;
          } else {
            z = wrapc(z);
          }
          kv[u] = v;
          bk[u] = bucket(x, y, z);
          kk[u] = local ? (int32_t)(pack_cell(x, y, z) ^ salt) : (int32_t)pack_cell(x, y, z);
        }
        const int first = kv[0] ? 0 : 1;  // cz itself is always valid
        const int last = kv[2] ? 2 : 1;
        bool consec = true;
        if (first == 0) consec = consec && bk[1] == bk[0] + 1;
        if (last == 2) consec = consec && bk[2] == bk[1] + 1;
        if (consec) {
          rb[pi] = (p == 0) ? q + 1 : bucket_start(loc, toff, first == 0 ? bk[0] : bk[1]);
          re[pi] = bucket_start(loc, toff, (last == 2 ? bk[2] : bk[1]) + 1);
          cen[pi] = (int32_t)pack_cell(x, y, cz);
          msk[pi] = (kv[0] ? 1 : 0) | 2 | (kv[2] ? 4 : 0);
        } else {
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            if (!kv[u]) continue;
            const bool only[3] = {u == 0, u == 1, u == 2};
            const int beg = (p == 0 && u == 1) ? q + 1 : bucket_start(loc, toff, bk[u]);
            const int end = bucket_start(loc, toff, bk[u] + 1);
            scan(beg, end, kk, only, dx, dy);
          }
        }
      }
      // phase 2: the consecutive-bucket pencils, four entries at a time
#pragma unroll
      for (int pi = 0; pi < NPT; ++pi) {
        const int p = g + pi * G;
        if (p >= N_PENCIL || rb[pi] >= re[pi]) continue;
        const int dx = p == 0 ? 0 : (p == 1 ? 0 : 1);
        const int dy = p == 0 ? 0 : (p == 1 ? 1 : p - 3);
        const T sx = (T)dx * hh, sy = (T)dy * hh;
        const uint32_t c0 = (uint32_t)cen[pi];
        const int mk = msk[pi];
        auto test2 = [&](const int2 e, const SBox<T>& b) {
          const uint32_t d = ((uint32_t)e.x ^ salt) - c0;
          int dz = 2;
          if (d == 0u) dz = 0;
          else if (d == (1u << 20)) dz = (mk & 4) ? 1 : 2;
          else if (d == (uint32_t)(-(1 << 20))) dz = (mk & 1) ? -1 : 2;
          const int m = e.y;
          if (dz != 2 && m != nk && m != pk && box_overlap(me, b, sx, sy, (T)dz * hh, tl))
            push(k, m);
        };
        const int end = re[pi];
        int q2 = rb[pi];
        for (; q2 + 4 <= end; q2 += 4) {
          int2 e4[4];
          SBox<T> b4[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            b4[v] = load_sbox<T>(sbox, q2 + v);
            e4[v] = entry_key_slot<SCR>(sent, b4[v], q2 + v);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) test2(e4[v], b4[v]);
        }
        for (; q2 < end; ++q2) {
          const SBox<T> b1 = load_sbox<T>(sbox, q2);
          test2(entry_key_slot<SCR>(sent, b1, q2), b1);
        }
      }
      if (g == 0) {
        // the element's box in global coordinates (any periodic image) for the
        // comparisons with large elements
        const double gh = local ? C.h : cs.h;
        const double go[3] = {local ? C.ox : 0.0, local ? C.oy : 0.0, local ? C.oz : 0.0};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          wl[i] = go[i] + ((double)(i == 0 ? cx : (i == 1 ? cy : cz)) * gh + (double)me.v[i]);
          ex[i] = (double)me.v[4 + i] - (double)me.v[i];
        }
        if constexpr (SCR == 1) {
          tlo = me.v[3];
          thi = me.v[7];
        } else {
          // the sorted entry holds key and slot there: the time range from the slot's box
          const float4* eb = (const float4*)ebox_slot + (size_t)k * 2;
          tlo = (double)eb[0].w + hc.tref;
          thi = (double)eb[1].w + hc.tref;
        }
      }
    } else {
      own_large = true;
      const LargeBox own = large[q - n_norm];
      k = own.slot;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        wl[i] = own.wl[i];
        ex[i] = own.ext[i];
      }
      tlo = own.tlo;
      thi = own.thi;
    }
    if (g == 0 && nl > 0) {
      const int nk = nxt[k], pk = prv[k];
      const int rk = rcell != nullptr ? rid[k] : 0;
      for (int a = 0; a < nl; ++a) {
        const LargeBox lb = large[a];
        const int m = lb.slot;
        if (m == k) continue;
        if (own_large && m < k) continue;
        if (m == nk || m == pk) continue;
        if (rcell != nullptr && rid[m] != rk) continue;  // another sub-region of the batch
        const double tt = hc.tol_t;
        bool ov = tlo <= lb.thi + tt && lb.tlo <= thi + tt;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          ov = ov && wrap_overlap(wl[i], ex[i], lb.wl[i], lb.ext[i], P, hc.tolL);
        if (ov) push(k, m);
      }
    }
  }
  __syncthreads();
  // staged candidates go out in one reservation once half the buffer is used, and after
  // the block's last chunk
  const int staged = s_cnt;
  if (staged >= SBUF_FLUSH || last) {
    const int cnt = min(staged, SBUF);
    if (threadIdx.x == 0 && cnt > 0) s_base = atomicAdd(&ctrl->n_cand, cnt);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += NT) {
      const int idx = s_base + i;
      if (idx < cap) cand[idx] = sbuf[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_cnt = 0;
  }
  __syncthreads();  // the buffer count is settled before the next chunk pushes
  }  // chunks
}

// The same half-shell screen, one element per thread, with the box tests spread evenly
// over the lanes of each wave. Every thread finds its element's five pencil ranges as
// k_screen does (phase 1). The wave then numbers the (element, entry) pairs of its 64
// elements in lane order (a scan of the per-element counts) and lane l takes pairs l,
// l + 64, ...: a wave runs ceil(pairs / 64) rounds, where one thread per element runs,
// for every pencil, as many rounds as its longest lane (about four times as many on the
// batched workload). A lane finds the element of its pair by a binary search over the
// wave's pair offsets and reads the element's box and ranges from the wave's LDS
// records; consecutive lanes then read consecutive entries of one range.
template <class T>
struct alignas(16) ScreenOwner {
  T lo[4];          // the element's box: low x, y, z; the cell edge
  T hi[4];          // high x, y, z; the slack
  int32_t k, nk, pk, salt;
  int32_t rbp[5];   // per pencil: its first entry minus the pairs before it
  int32_t pre[4];   // pairs before pencils 1..4
  int32_t cell, msk;  // the element's cell (unsalted), 3 valid-cell bits per pencil
  int32_t pad;
};
constexpr int SBUF_FLAT = 960;       // staged candidates per block (LDS shared with the records)
constexpr int SBUF_FLAT_FLUSH = 480;

template <int SCR>
__global__ __launch_bounds__(NT, SCR == 2 ? 5 : 1) void k_screen_flat(
    int n, const int2* __restrict__ sent, const void* __restrict__ sbox,
    const void* __restrict__ ebox_slot, const int32_t* __restrict__ nxt,
    const int32_t* __restrict__ prv, const int32_t* __restrict__ loc,
    const int32_t* __restrict__ toff, int ntiles, const LargeBox* __restrict__ large, HashCfg hc,
    sp::Period P, int2* __restrict__ cand, int cap, Ctrl* ctrl, const int32_t* __restrict__ rid,
    const RCell* __restrict__ rcell) {
  if (ctrl->done) return;
  using T = typename std::conditional<SCR == 1, double, float>::type;
  static_assert(sizeof(ScreenOwner<T>) % 16 == 0, "records are read as 16-byte vectors");
  __shared__ int2 sbuf[SBUF_FLAT];
  __shared__ ScreenOwner<T> s_own[NT];
  __shared__ int s_cnt, s_base;
  const Cells cs = ctrl->cells;
  const int nl = ctrl->n_large;
  const int n_norm = toff[ntiles];
  const bool local = rcell != nullptr;
  const int nchunk = (n_norm + nl + NT - 1) / NT;
  const int cper = (nchunk + N_XCD - 1) / N_XCD;
  const int xcd = (int)blockIdx.x % N_XCD;
  const int bper = (int)gridDim.x / N_XCD;
  const int lane = (int)(threadIdx.x & 63);
  const int wbase = (int)threadIdx.x - lane;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  for (int c = (int)blockIdx.x / N_XCD; c < cper; c += bper) {
  const int lid = xcd * cper + c;
  if (lid >= nchunk) break;
  const bool last = c + bper >= cper || lid + bper >= nchunk;
  const int q = lid * NT + (int)threadIdx.x;
  auto push = [&](int a, int b) {
    const int i = atomicAdd(&s_cnt, 1);
    if (i < SBUF_FLAT)
      sbuf[i] = make_int2(a, b);
    else
      push_cand(ctrl, cand, cap, a, b);
  };
  int npairs = 0;
  int k = -1;
  bool own_large = false;
  double wl[3], ex[3], tlo = 0.0, thi = 0.0;  // a large element's wrapped box
  if (q < n_norm) {
    // phase 1: the element, its grid and its five pencil ranges
    const SBox<T> me = load_sbox<T>(sbox, q);
    const int2 ent = entry_key_slot<SCR>(sent, me, q);
    k = ent.y;
    RCell C{};
    uint32_t salt = 0;
    int gnc = cs.nc;
    if (local) {
      C = rcell[rid[k]];
      salt = C.salt;
      gnc = C.nc;
    }
    const int32_t cc = (int32_t)((uint32_t)ent.x ^ salt);
    const int nk = nxt[k], pk = prv[k];
    const int cx = cc & 1023, cy = (cc >> 10) & 1023, cz = (cc >> 20) & 1023;
    const T tl = SCR == 1 ? (T)hc.tol : (T)(local ? C.marg32 : cs.marg32);
    const T hh = SCR == 1 ? (T)(local ? C.h : cs.h) : (T)(local ? C.h32 : cs.h32);
    auto bucket = [&](int x, int y, int z) -> uint32_t {
      return local ? (C.base + cell_index(gnc, x, y, z)) & hc.bmask
                   : bucket_of(gnc, hc.bmask, x, y, z);
    };
    auto wrapc = [&](int v) { return v < 0 ? v + gnc : (v >= gnc ? v - gnc : v); };
    // cells whose buckets are not consecutive (rare): tested here, one entry at a time
    auto scan_cell = [&](int beg, int end, int32_t key, int dx, int dy, int dz) {
      const T sx = (T)dx * hh, sy = (T)dy * hh, sz = (T)dz * hh;
      for (int q2 = beg; q2 < end; ++q2) {
        const SBox<T> b = load_sbox<T>(sbox, q2);
        const int2 e = entry_key_slot<SCR>(sent, b, q2);
        const int m = e.y;
        if (e.x == key && m != nk && m != pk && box_overlap(me, b, sx, sy, sz, tl)) push(k, m);
      }
    };
    // cells one step up an axis that the element cannot reach are not read
    bool up[3];
    reach_up(me, hh, tl, hc.tol, up);
    int rb[N_PENCIL], len[N_PENCIL], msk = 0;
#pragma unroll
    for (int p = 0; p < N_PENCIL; ++p) {
      rb[p] = 0;
      len[p] = 0;
      const int dx = p < 2 ? 0 : 1;
      const int dy = p == 0 ? 0 : (p == 1 ? 1 : p - 3);
      if ((dx == 1 && !up[0]) || (dy == 1 && !up[1])) continue;
      int x = cx + dx, y = cy + dy;
      if (local) {
        if (x >= gnc || y < 0 || y >= gnc) continue;
      } else {
        x = wrapc(x);
        y = wrapc(y);
      }
      bool kv[3];
      uint32_t bk[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int dz = u - 1;
        int z = cz + dz;
        bool v = !(p == 0 && dz < 0) && (dz < 1 || up[2]);
        if (local) {
          v = v && z >= 0 && z < gnc;
        } else {
          z = wrapc(z);
        }
        kv[u] = v;
        bk[u] = bucket(x, y, z);
      }
      const int first = kv[0] ? 0 : 1;
      const int lst = kv[2] ? 2 : 1;
      bool consec = true;
      if (first == 0) consec = consec && bk[1] == bk[0] + 1;
      if (lst == 2) consec = consec && bk[2] == bk[1] + 1;
      if (consec) {
        rb[p] = (p == 0) ? q + 1 : bucket_start(loc, toff, first == 0 ? bk[0] : bk[1]);
        len[p] = max(0, bucket_start(loc, toff, (lst == 2 ? bk[2] : bk[1]) + 1) - rb[p]);
        msk |= ((kv[0] ? 1 : 0) | 2 | (kv[2] ? 4 : 0)) << (3 * p);
      } else {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          if (!kv[u]) continue;
          int z = cz + u - 1;
          if (!local) z = wrapc(z);
          const int32_t key =
              local ? (int32_t)(pack_cell(x, y, z) ^ salt) : (int32_t)pack_cell(x, y, z);
          const int beg = (p == 0 && u == 1) ? q + 1 : bucket_start(loc, toff, bk[u]);
          scan_cell(beg, bucket_start(loc, toff, bk[u] + 1), key, dx, dy, u - 1);
        }
      }
    }
    // the wave's LDS record of this element
    ScreenOwner<T>& w = s_own[threadIdx.x];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      w.lo[i] = me.v[i];
      w.hi[i] = me.v[4 + i];
    }
    w.lo[3] = hh;
    w.hi[3] = tl;
    w.k = k;
    w.nk = nk;
    w.pk = pk;
    w.salt = (int32_t)salt;
    int acc = 0;
#pragma unroll
    for (int p = 0; p < N_PENCIL; ++p) {
      if (p > 0) w.pre[p - 1] = acc;
      w.rbp[p] = rb[p] - acc;
      acc += len[p];
    }
    w.cell = (int32_t)pack_cell(cx, cy, cz);
    w.msk = msk;
    npairs = acc;
  } else if (q < n_norm + nl) {
    own_large = true;
    const LargeBox own = large[q - n_norm];
    k = own.slot;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      wl[i] = own.wl[i];
      ex[i] = own.ext[i];
    }
    tlo = own.tlo;
    thi = own.thi;
  }
  // phase 2: the wave's pairs in lane order, two rounds of 64 per pass
  int incl = npairs;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  const int off = incl - npairs;
  const int total = __shfl(incl, 63, 64);
  __syncthreads();  // the records are written
  for (int base = 0; base < total; base += 128) {
    int pia[2], oa[2], qa[2];
    SBox<T> ba[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int p = base + 64 * u + lane;
      // the element of pair p: the last lane whose first pair is at or before p
      int o = 0, oo = 0;
#pragma unroll
      for (int st = 32; st > 0; st >>= 1) {
        const int oc = __shfl(off, o + st, 64);
        if (oc <= p) {
          o += st;
          oo = oc;
        }
      }
      pia[u] = 0;
      oa[u] = o;
      qa[u] = -1;
      if (p < total) {
        const ScreenOwner<T>& w = s_own[wbase + o];
        const int r = p - oo;
        const int pi = (r >= w.pre[0]) + (r >= w.pre[1]) + (r >= w.pre[2]) + (r >= w.pre[3]);
        pia[u] = pi;
        qa[u] = w.rbp[pi] + r;
        ba[u] = load_sbox<T>(sbox, qa[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (qa[u] < 0) continue;
      const ScreenOwner<T>& w = s_own[wbase + oa[u]];
      const int pi = pia[u];
      const int dx = pi < 2 ? 0 : 1;
      const int dy = pi == 0 ? 0 : (pi == 1 ? 1 : pi - 3);
      const int32_t wc = w.cell;
      int x = (wc & 1023) + dx, y = ((wc >> 10) & 1023) + dy;
      if (!local) {
        const int gnc = cs.nc;
        x = x >= gnc ? x - gnc : x;
        y = y < 0 ? y + gnc : (y >= gnc ? y - gnc : y);
      }
      const uint32_t c0 = pack_cell(x, y, (wc >> 20) & 1023);
      const int mk = (w.msk >> (3 * pi)) & 7;
      const int2 e = entry_key_slot<SCR>(sent, ba[u], qa[u]);
      const uint32_t d = ((uint32_t)e.x ^ (uint32_t)w.salt) - c0;
      int dz = 2;
      if (d == 0u) dz = 0;
      else if (d == (1u << 20)) dz = (mk & 4) ? 1 : 2;
      else if (d == (uint32_t)(-(1 << 20))) dz = (mk & 1) ? -1 : 2;
      const int m = e.y;
      if (dz != 2 && m != w.nk && m != w.pk) {
        SBox<T> me;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          me.v[i] = w.lo[i];
          me.v[4 + i] = w.hi[i];
        }
        const T hh = w.lo[3];
        if (box_overlap(me, ba[u], (T)dx * hh, (T)dy * hh, (T)dz * hh, w.hi[3])) push(w.k, m);
      }
    }
  }
  // two large elements: tested by the one of smaller slot (large against hashed ones:
  // k_screen_large)
  if (own_large && nl > 0) {
    const int nk = nxt[k], pk = prv[k];
    const int rk = local ? rid[k] : 0;
    for (int a = 0; a < nl; ++a) {
      const LargeBox lb = large[a];
      const int m = lb.slot;
      if (m == k) continue;
      if (own_large && m < k) continue;
      if (m == nk || m == pk) continue;
      if (local && rid[m] != rk) continue;  // another sub-region of the batch
      const double tt = hc.tol_t;
      bool ov = tlo <= lb.thi + tt && lb.tlo <= thi + tt;
#pragma unroll
      for (int i = 0; i < 3; ++i)
        ov = ov && wrap_overlap(wl[i], ex[i], lb.wl[i], lb.ext[i], P, hc.tolL);
      if (ov) push(k, m);
    }
  }
  __syncthreads();
  // staged candidates go out in one reservation once half the buffer is used, and after
  // the block's last chunk
  const int staged = s_cnt;
  if (staged >= SBUF_FLAT_FLUSH || last) {
    const int cnt = min(staged, SBUF_FLAT);
    if (threadIdx.x == 0 && cnt > 0) s_base = atomicAdd(&ctrl->n_cand, cnt);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += NT) {
      const int idx = s_base + i;
      if (idx < cap) cand[idx] = sbuf[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_cnt = 0;
  }
  __syncthreads();  // the buffer count and the records are free for the next chunk
  }  // chunks
}

// Large elements against the hashed ones, for the screen that leaves those pairs out
// (k_screen_flat): one wave per large element walks the grid cells its box can reach
// (every hashed element lies in the cell of its lower corner, clamped to the grid, and
// spans less than a cell, so an overlapping one has its corner in [lo - h, hi] per
// axis), a lane per cell, and tests that cell's entries in the frame of the element's
// grid: the local grid of its sub-region (clamped cells) or the periodic box's (cells
// wrapped). Spatial test with the large-element slack; the exact 4-D test follows in
// k_confirm. Each (large, hashed) pair is seen once: the hashed element sits in one cell.
template <int SCR>
__global__ __launch_bounds__(NT) void k_screen_large(
    const int2* __restrict__ sent, const void* __restrict__ sbox,
    const int32_t* __restrict__ nxt, const int32_t* __restrict__ prv,
    const int32_t* __restrict__ loc, const int32_t* __restrict__ toff,
    int ntiles, const LargeBox* __restrict__ large, HashCfg hc, sp::Period P,
    int2* __restrict__ cand, int cap, Ctrl* ctrl, const int32_t* __restrict__ rid,
    const RCell* __restrict__ rcell) {
  if (ctrl->done) return;
  const int n_norm = toff[ntiles];
  using T = typename std::conditional<SCR == 1, double, float>::type;
  const int nl = ctrl->n_large;
  const Cells cs = ctrl->cells;
  const bool local = rcell != nullptr;
  if (!local && cs.nc == 0) return;  // no grid: every element is large
  const int lane = (int)(threadIdx.x & 63);
  const int nwave = (int)(gridDim.x * (NT / 64));
  for (int a = (int)(blockIdx.x * (NT / 64) + (threadIdx.x >> 6)); a < nl; a += nwave) {
    const LargeBox L = large[a];
    const int k = L.slot;
    const int nk = nxt[k], pk = prv[k];
    RCell C{};
    int nc = cs.nc;
    double h = cs.h, inv_h = cs.inv_h;
    uint32_t salt = 0;
    double lo[3];  // the element's lower corner in the grid's frame
    if (local) {
      C = rcell[rid[k]];
      nc = C.nc;
      h = C.h;
      inv_h = C.inv_h;
      salt = C.salt;
      const double o[3] = {C.ox, C.oy, C.oz};
      const double half = 0.5 * (double)nc * h;  // the image nearest the grid's centre
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double d = L.wl[c] - o[c];
        lo[c] = d - P.box * P.nearest(d - half);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) lo[c] = L.wl[c];
    }
    // cell range per axis; a wrapped range of nc or more cells is the whole axis
    int c0[3], cn[3];
    int total = 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int a0 = (int)floor((lo[c] - h - hc.tolL) * inv_h);
      int a1 = (int)floor((lo[c] + L.ext[c] + hc.tolL) * inv_h);
      if (local) {
        a0 = a0 < 0 ? 0 : (a0 > nc - 1 ? nc - 1 : a0);
        a1 = a1 < 0 ? 0 : (a1 > nc - 1 ? nc - 1 : a1);
      } else if (a1 - a0 + 1 >= nc) {
        a0 = 0;
        a1 = nc - 1;
      }
      c0[c] = a0;
      cn[c] = a1 - a0 + 1;
      total *= cn[c];
    }
    // entry q2 of cell cc against the element
    auto test = [&](int q2, const int (&cc)[3], int32_t key, bool check_region) {
      const SBox<T> e = load_sbox<T>(sbox, q2);
      const int2 ks = entry_key_slot<SCR>(sent, e, q2);
      const int m = ks.y;
      if (ks.x != key || m == k || m == nk || m == pk) return;
      if (check_region && rid[m] != rid[k]) return;
      bool ov = true;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double elo = (double)cc[c] * h + (double)e.v[c];
        const double eex = (double)e.v[4 + c] - (double)e.v[c];
        if (local)
          ov = ov && elo <= lo[c] + L.ext[c] + hc.tolL && lo[c] <= elo + eex + hc.tolL;
        else
          ov = ov && wrap_overlap(lo[c], L.ext[c], elo, eex, P, hc.tolL);
      }
      if (ov) push_cand(ctrl, cand, cap, k, m);
    };
    if (total <= LARGE_CELLS) {
      for (int i = lane; i < total; i += 64) {
        int cc[3] = {c0[0] + i % cn[0], c0[1] + (i / cn[0]) % cn[1], c0[2] + i / (cn[0] * cn[1])};
        if (!local)
#pragma unroll
          for (int c = 0; c < 3; ++c) cc[c] = ((cc[c] % nc) + nc) % nc;
        const uint32_t b = local ? (C.base + cell_index(nc, cc[0], cc[1], cc[2])) & hc.bmask
                                 : bucket_of(nc, hc.bmask, cc[0], cc[1], cc[2]);
        const int32_t key = (int32_t)(pack_cell(cc[0], cc[1], cc[2]) ^ salt);
        const int beg = bucket_start(loc, toff, b), end = bucket_start(loc, toff, b + 1);
        for (int q2 = beg; q2 < end; ++q2) test(q2, cc, key, false);
      }
    } else {
      // an element reaching more cells than there are worth visiting (cells much smaller
      // than it, e.g. a fixed small cell size): every hashed entry of its region instead,
      // its cell read from its key
      for (int q2 = lane; q2 < n_norm; q2 += 64) {
        const int2 ks = sent_key_slot<SCR>(sent, sbox, q2);
        const uint32_t u = (uint32_t)ks.x ^ salt;
        const int cc[3] = {(int)(u & 1023), (int)((u >> 10) & 1023), (int)((u >> 20) & 1023)};
        test(q2, cc, ks.x, local);
      }
    }
  }
}

// The same half-shell screen, one thread per element, with the five pencil ranges read
// from the element's PencilAux (written by k_scatter) instead of being looked up here:
// a thread loads its entry and its 64-byte record, then scans its pencils. Pencils whose
// cells are not consecutive buckets, and the tests against large elements, read the
// element's grid and look their cells up as k_screen does.
template <int SCR>
__global__ __launch_bounds__(NT, 5) void k_screen_pre(int n, const int2* __restrict__ sent,
                                                   const void* __restrict__ sbox,
                                                   const void* __restrict__ ebox_slot,
                                                   const PencilAux* __restrict__ saux,
                                                   const int32_t* __restrict__ loc,
                                                   const int32_t* __restrict__ toff, int ntiles,
                                                   const LargeBox* __restrict__ large, HashCfg hc,
                                                   sp::Period P, int2* __restrict__ cand, int cap,
                                                   Ctrl* ctrl, const int32_t* __restrict__ rid,
                                                   const RCell* __restrict__ rcell,
                                                   const int32_t* __restrict__ nxt,
                                                   const int32_t* __restrict__ prv) {
  if (ctrl->done) return;
  using T = typename std::conditional<SCR == 1, double, float>::type;
  __shared__ int2 sbuf[SBUF];
  __shared__ int s_cnt, s_base;
  const Cells cs = ctrl->cells;
  const int nl = ctrl->n_large;
  const int n_norm = toff[ntiles];
  const int nchunk = (n_norm + nl + NT - 1) / NT;
  const int cper = (nchunk + N_XCD - 1) / N_XCD;
  const int xcd = (int)blockIdx.x % N_XCD;
  const int bper = (int)gridDim.x / N_XCD;
  const bool local = rcell != nullptr;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  for (int c = (int)blockIdx.x / N_XCD; c < cper; c += bper) {
  const int lid = xcd * cper + c;
  if (lid >= nchunk) break;
  const bool last = c + bper >= cper || lid + bper >= nchunk;
  const int q = lid * NT + (int)threadIdx.x;
  auto push = [&](int a, int b) {
    const int i = atomicAdd(&s_cnt, 1);
    if (i < SBUF)
      sbuf[i] = make_int2(a, b);
    else
      push_cand(ctrl, cand, cap, a, b);
  };
  if (q < n_norm + nl) {
    int k, nk, pk;
    bool own_large;
    double wl[3], ex[3], tlo, thi;  // wrapped box of the element (for large partners)
    if (q < n_norm) {
      own_large = false;
      const SBox<T> me = load_sbox<T>(sbox, q);
      const int2 ent = entry_key_slot<SCR>(sent, me, q);
      const PencilAux A = saux[q];
      k = ent.y;
      nk = A.nk;
      pk = A.pk;
      const uint32_t salt = A.salt;
      const int32_t cc = (int32_t)((uint32_t)ent.x ^ salt);
      const int cx = cc & 1023, cy = (cc >> 10) & 1023, cz = (cc >> 20) & 1023;
      const T tl = SCR == 1 ? (T)hc.tol : (T)A.marg32;
      // FP64 boxes are relative to a cell edge of FP64 precision (the grid's own h)
      T hh;
      if constexpr (SCR == 1) hh = (T)(local ? rcell[rid[k]].h : cs.h);
      else hh = (T)A.h32;
      const int gnc = cs.nc;  // the periodic grid's size (a batch's grids do not wrap)
      auto wrapc = [&](int v) { return v < 0 ? v + gnc : (v >= gnc ? v - gnc : v); };
      auto test_range = [&](int beg, int end, uint32_t c0, int mk, int dx, int dy) {
        const T sx = (T)dx * hh, sy = (T)dy * hh;
        auto test2 = [&](const int2 e, const SBox<T>& b) {
          const uint32_t d = ((uint32_t)e.x ^ salt) - c0;
          int dz = 2;
          if (d == 0u) dz = 0;
          else if (d == (1u << 20)) dz = (mk & 4) ? 1 : 2;
          else if (d == (uint32_t)(-(1 << 20))) dz = (mk & 1) ? -1 : 2;
          const int m = e.y;
          if (dz != 2 && m != nk && m != pk && box_overlap(me, b, sx, sy, (T)dz * hh, tl))
            push(k, m);
        };
        int q2 = beg;
        for (; q2 + 4 <= end; q2 += 4) {
          int2 e4[4];
          SBox<T> b4[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            b4[v] = load_sbox<T>(sbox, q2 + v);
            e4[v] = entry_key_slot<SCR>(sent, b4[v], q2 + v);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) test2(e4[v], b4[v]);
        }
        for (; q2 < end; ++q2) {
          const SBox<T> b1 = load_sbox<T>(sbox, q2);
          test2(entry_key_slot<SCR>(sent, b1, q2), b1);
        }
      };
      const uint32_t msk = A.msk;
#pragma unroll
      for (int p = 0; p < N_PENCIL; ++p) {
        const int mk = (int)((msk >> (3 * p)) & 7u);
        if (!mk) continue;  // the row lies outside the region's grid
        int dx, dy;
        pencil_offsets(p, dx, dy);
        const int x = local ? cx + dx : wrapc(cx + dx);
        const int y = local ? cy + dy : wrapc(cy + dy);
        if ((msk >> (15 + p)) & 1u) {
          // cells that are not consecutive buckets (a wrap in z, the end of the bucket
          // table): each valid cell looked up alone
          RCell C{};
          if (local) C = rcell[rid[k]];
          const int lnc = local ? C.nc : gnc;
          const T sx = (T)dx * hh, sy = (T)dy * hh;
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            if (!((mk >> u) & 1)) continue;
            const int z = local ? cz + u - 1 : wrapc(cz + u - 1);
            const uint32_t bk = local ? (C.base + cell_index(lnc, x, y, z)) & hc.bmask
                                      : bucket_of(lnc, hc.bmask, x, y, z);
            const int beg = (p == 0 && u == 1) ? q + 1 : bucket_start(loc, toff, bk);
            const int end = bucket_start(loc, toff, bk + 1);
            // entries of this one cell (others share its bucket), shifted by u - 1 cells
            const int32_t kk = (int32_t)(pack_cell(x, y, z) ^ salt);
            const T sz = (T)(u - 1) * hh;
            for (int q2 = beg; q2 < end; ++q2) {
              const SBox<T> b1 = load_sbox<T>(sbox, q2);
              const int2 e = entry_key_slot<SCR>(sent, b1, q2);
              const int m = e.y;
              if (e.x == kk && m != nk && m != pk && box_overlap(me, b1, sx, sy, sz, tl))
                push(k, m);
            }
          }
          continue;
        }
        const int beg = p == 0 ? q + 1 : A.rb[p - 1];
        const int end = p == 0 ? A.re0 : A.re[p - 1];
        test_range(beg, end, pack_cell(x, y, cz), mk, dx, dy);
      }
      if (nl > 0) {
        // the element's box in global coordinates (any periodic image) for the
        // comparisons with large elements
        RCell C{};
        if (local) C = rcell[rid[k]];
        const double gh = local ? C.h : cs.h;
        const double go[3] = {local ? C.ox : 0.0, local ? C.oy : 0.0, local ? C.oz : 0.0};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          wl[i] = go[i] + ((double)(i == 0 ? cx : (i == 1 ? cy : cz)) * gh + (double)me.v[i]);
          ex[i] = (double)me.v[4 + i] - (double)me.v[i];
        }
        if constexpr (SCR == 1) {
          tlo = me.v[3];
          thi = me.v[7];
        } else {
          const float4* eb = (const float4*)ebox_slot + (size_t)k * 2;
          tlo = (double)eb[0].w + hc.tref;
          thi = (double)eb[1].w + hc.tref;
        }
      }
    } else {
      own_large = true;
      const LargeBox own = large[q - n_norm];
      k = own.slot;
      nk = nxt[k];
      pk = prv[k];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        wl[i] = own.wl[i];
        ex[i] = own.ext[i];
      }
      tlo = own.tlo;
      thi = own.thi;
    }
    if (nl > 0) {
      const int rk = rcell != nullptr ? rid[k] : 0;
      for (int a = 0; a < nl; ++a) {
        const LargeBox lb = large[a];
        const int m = lb.slot;
        if (m == k) continue;
        if (own_large && m < k) continue;
        if (m == nk || m == pk) continue;
        if (rcell != nullptr && rid[m] != rk) continue;  // another sub-region of the batch
        const double tt = hc.tol_t;
        bool ov = tlo <= lb.thi + tt && lb.tlo <= thi + tt;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          ov = ov && wrap_overlap(wl[i], ex[i], lb.wl[i], lb.ext[i], P, hc.tolL);
        if (ov) push(k, m);
      }
    }
  }
  __syncthreads();
  const int staged = s_cnt;
  if (staged >= SBUF_FLUSH || last) {
    const int cnt = min(staged, SBUF);
    if (threadIdx.x == 0 && cnt > 0) s_base = atomicAdd(&ctrl->n_cand, cnt);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += NT) {
      const int idx = s_base + i;
      if (idx < cap) cand[idx] = sbuf[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_cnt = 0;
  }
  __syncthreads();
  }  // chunks
}

__device__ __forceinline__ Elem load_elem(const Slices& X, int ic, int in, int a, int ja,
                                          const sp::Period& P) {
  return sp::make_elem(ld(X, ic, a), ld(X, ic, ja), ld(X, in, a), ld(X, in, ja), P);
}

// Exact FP64 box overlap and the four triangle pairs of each candidate.
__global__ __launch_bounds__(NT) void k_confirm(Slices X, const int32_t* __restrict__ nxt,
                                                const int64_t* __restrict__ id, sp::Period P,
                                                const int2* __restrict__ cand, int cap_cand,
                                                EvCand* __restrict__ ev, int cap_evt, Ctrl* ctrl) {
  if (ctrl->done) return;
  const int nc = min(ctrl->n_cand, cap_cand);
  const int s = ctrl->step;
  const int ic = s % 3, in = (s + 1) % 3;
  for (int i = blockIdx.x * NT + threadIdx.x; i < nc; i += gridDim.x * NT) {
    const int2 pr = cand[i];
    int a = pr.x, b = pr.y;
    int64_t ia = id[a], ib = id[b];
    if (ib < ia) {
      const int tmp = a;
      a = b;
      b = tmp;
      const int64_t ti = ia;
      ia = ib;
      ib = ti;
    }
    const Elem ea = load_elem(X, ic, in, a, nxt[a], P);
    Elem eb = load_elem(X, ic, in, b, nxt[b], P);
    const Box4 ba = sp::elem_box(ea);
    const Box4 bb = sp::elem_box(eb);
    const V4 Aa = ea.v[0], Ab = eb.v[0];
    const double S[3] = {P.box * P.nearest(Ab.x - Aa.x), P.box * P.nearest(Ab.y - Aa.y),
                         P.box * P.nearest(Ab.z - Aa.z)};
    bool ov = true;
    for (int c = 0; c < 3; ++c)
      ov = ov && (ba.lo[c] <= bb.hi[c] - S[c]) && (bb.lo[c] - S[c] <= ba.hi[c]);
    ov = ov && (ba.lo[3] <= bb.hi[3]) && (bb.lo[3] <= ba.hi[3]);
    if (!ov) continue;
    for (int v = 0; v < 4; ++v) {
      eb.v[v].x = eb.v[v].x - S[0];
      eb.v[v].y = eb.v[v].y - S[1];
      eb.v[v].z = eb.v[v].z - S[2];
    }
    bool found = false;
    double bt = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
    for (int ipq = 0; ipq < 4; ++ipq) {
      const int ipp = ipq >> 1, iq = ipq & 1;
      const V4& P0 = ipp ? ea.v[2] : ea.v[0];
      const V4& P1 = ea.v[1];
      const V4& P2 = ipp ? ea.v[3] : ea.v[2];
      const V4& Q0 = iq ? eb.v[2] : eb.v[0];
      const V4& Q1 = eb.v[1];
      const V4& Q2 = iq ? eb.v[3] : eb.v[2];
      double t, x, y, z;
      if (sp::tri_tri(P0, P1, P2, Q0, Q1, Q2, t, x, y, z)) {
        if (!found || t < bt) {
          found = true;
          bt = t;
          bx = x;
          by = y;
          bz = z;
        }
      }
    }
    if (!found) continue;
    const int e = atomicAdd(&ctrl->n_evt, 1);
    if (e < cap_evt) {
      EvCand c;
      c.t = bt;
      c.ida = ia;
      c.idb = ib;
      c.sa = a;
      c.sb = b;
      c.x = bx;
      c.y = by;
      c.z = bz;
      ev[e] = c;
    }
  }
}

// The draw that decides whether a crossing exchanges partners (Section "Semi-parallel
// cosmic string simulation": with probability p). Philox4x64-10 (Salmon, Moraes, Dror and
// Shaw, SC 2011) under key (seed, 0) of counter (id_a, id_b, step, 0): per round the
// products M0 c0 and M1 c2 give (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0), then the key
// advances by the Weyl increments. u = (word 0 >> 11) 2^-53, an exact FP64 value in [0, 1).
__device__ __forceinline__ double crossing_draw(uint64_t seed, int32_t step, int64_t ida,
                                                int64_t idb) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  uint64_t c0 = (uint64_t)ida, c1 = (uint64_t)idb, c2 = (uint64_t)(int64_t)step, c3 = 0;
  uint64_t k0 = seed, k1 = 0;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B97F4A7C15ull;
    k1 += 0xBB67AE8584CAA73Bull;
  }
  return (double)(c0 >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ bool key_less(const EvCand& p, const EvCand& q) {
  if (p.t < q.t) return true;
  if (p.t > q.t) return false;
  if (p.ida != q.ida) return p.ida < q.ida;
  return p.idb < q.idb;
}

__device__ __forceinline__ uint64_t aload64(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t aload32(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore32(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claim `slot` for event e in iteration `st` unless an event of smaller key holds it.
__device__ __forceinline__ void propose(uint64_t* best, int slot, uint32_t st, int e,
                                       const EvCand* ev) {
  const uint64_t tag = ((uint64_t)st << 32) | (uint32_t)e;
  uint64_t old = aload64(&best[slot]);
  for (;;) {
    if ((uint32_t)(old >> 32) == st) {
      const int oe = (int)(uint32_t)old;
      if (key_less(ev[oe], ev[e])) return;
    }
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&best[slot], (unsigned long long)old, (unsigned long long)tag);
    if (prev == old) return;
    old = prev;
  }
}

// Matching in LDS (groups with at most RES_LDS_EVT events): each event's two elements get
// a local index through an open-addressing table of slots, and a round's proposals are
// LDS atomics on 32-bit tags (round << 12 | local event). A slot taken by an accepted
// event holds RES_USED. Key comparisons use the bits of t* (order-preserving) and fall
// back to the ids in global memory only on equal t*.
constexpr int RES_LDS_EVT = 3072;
constexpr int RES_HASH = 12288;  // > 2 RES_LDS_EVT: an insert always finds room
constexpr uint32_t RES_USED = 0xFFFFFFFFu;
constexpr int RES_GROUPS = 32;   // most workgroups of the matching (batches)
static_assert(RES_LDS_EVT <= 4096, "event index in the low 12 bits of a tag");

__device__ __forceinline__ uint64_t order_bits(double t) {
  const uint64_t u = (uint64_t)__double_as_longlong(t + 0.0);  // -0 -> +0
  return (u >> 63) ? ~u : (u | (1ull << 63));
}

// Local event i's key is below local event j's: (t*, id_a, id_b) order.
__device__ __forceinline__ bool lkey_less(const uint64_t* s_t, const int32_t* s_list,
                                          const EvCand* ev, int i, int j) {
  const uint64_t a = s_t[i], b = s_t[j];
  if (a != b) return a < b;
  const EvCand& e = ev[s_list[i]];
  const EvCand& f = ev[s_list[j]];
  if (e.ida != f.ida) return e.ida < f.ida;
  return e.idb < f.idb;
}

// Local index of `slot` in the table (inserted if absent).
__device__ __forceinline__ int lslot(int32_t* s_hkey, int32_t slot) {
  uint32_t h = (uint32_t)(((uint64_t)((uint32_t)slot * 0x9E3779B1u) * RES_HASH) >> 32);
  for (;;) {
    const int32_t prev = atomicCAS(&s_hkey[h], -1, slot);
    if (prev == -1 || prev == slot) return (int)h;
    h = h + 1 == (uint32_t)RES_HASH ? 0u : h + 1;
  }
}

// Claim local slot h for local event i with `tag` unless an event of smaller key holds it
// this round, or an accepted event took it.
__device__ __forceinline__ void lpropose(uint32_t* s_best, int h, uint32_t tag, int i,
                                         const uint64_t* s_t, const int32_t* s_list,
                                         const EvCand* ev) {
  uint32_t old = __hip_atomic_load(&s_best[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  for (;;) {
    if (old == RES_USED) return;
    if ((old >> 12) == (tag >> 12) && lkey_less(s_t, s_list, ev, (int)(old & 4095u), i)) return;
    const uint32_t prev = atomicCAS(&s_best[h], old, tag);
    if (prev == old) return;
    old = prev;
  }
}

// Each sub-region's local grid for the next step (h_set > 0: that cell edge; else grow
// x its largest element extent of this step), and the bucket bases (prefix sums of the
// grids' cell counts). Called by a whole workgroup of 1024 threads; s_sum holds 1024
// values of LDS.
__device__ __forceinline__ void rcells_update(const RegionGeom* __restrict__ geoms, int n_sub,
                                              uint64_t* __restrict__ rext,
                                              RCell* __restrict__ rc, double h_set,
                                              const Ctrl* ctrl, uint64_t* s_sum) {
  const int t = threadIdx.x;
  const int per = (n_sub + 1023) / 1024;
  const double grow = ctrl->grow;
  uint64_t sum = 0;
  for (int i = 0; i < per; ++i) {
    const int q = t * per + i;
    if (q >= n_sub) break;
    RCell C = rc[q];
    const double g = 0.5 / geoms[q].inv2g;
    const double W = RCELL_W * g;
    double target = h_set;
    if (h_set <= 0.0) {
      const uint64_t x = rext[(size_t)q * REXT_STRIDE];
      target = x != 0 ? grow * from_key(x) : (C.nc > 0 ? C.h : W / 3.0);
    }
    rext[(size_t)q * REXT_STRIDE] = 0;
    int nc = (int)floor(W / target);
    nc = nc < 3 ? 3 : (nc > 1023 ? 1023 : nc);
    C.nc = nc;
    C.h = W / nc;
    C.inv_h = 1.0 / C.h;
    C.hlim = C.h - 4.0 * ctrl->tol;
    C.h32 = (float)C.h;
    // FP32 slack: a few ulps at the largest local magnitude (clamped elements lie up to
    // W from a cell origin)
    C.marg32 = (float)((W + 3.0 * C.h) * 0x1p-20);
    double ctr[3];
    region_centre(geoms[q], ctr);
    C.ox = ctr[0] - 0.5 * W;
    C.oy = ctr[1] - 0.5 * W;
    C.oz = ctr[2] - 0.5 * W;
    C.salt = (uint32_t)q * 0x9E3779B1u;
    rc[q] = C;
    sum += cell_count(nc);
  }
  s_sum[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint64_t add = t >= o ? s_sum[t - o] : 0;
    __syncthreads();
    s_sum[t] += add;
    __syncthreads();
  }
  uint64_t run = s_sum[t] - sum;
  for (int i = 0; i < per; ++i) {
    const int q = t * per + i;
    if (q >= n_sub) break;
    rc[q].base = (uint32_t)run;
    run += cell_count(rc[q].nc);
  }
}

// Wave-aggregated reservation: lanes with `want` get consecutive places from one
// atomicAdd on *ctr per wave; returns this lane's place (or -1).
__device__ __forceinline__ int wave_reserve(int32_t* ctr, bool want) {
  const uint64_t m = __ballot(want);
  if (!m) return -1;
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((unsigned long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(ctr, __popcll(m));
  base = __shfl(base, leader, 64);
  const uint64_t below = lane == 0 ? 0ull : (m & (~0ull >> (64 - lane)));
  return want ? base + __popcll(below) : -1;
}

// The greedy matching of the step's events in (t*, id_a, id_b) order, computed as
// iterated local minima; partner exchange; log; step bookkeeping. Events of different
// sub-regions of a batch never share an element, so each workgroup takes the events of
// the sub-regions q with q mod gridDim.x == blockIdx.x and matches them alone (one
// workgroup for a single region). With p < 1 each crossing first draws u; one with
// u >= p passes through: it is logged (kind 1) and marks its elements for the loop rule,
// but claims neither. The last workgroup to finish does the step's bookkeeping.
__global__ __launch_bounds__(RESOLVE_NT) void k_resolve(
    int32_t* __restrict__ nxt, int32_t* __restrict__ prv, const EvCand* __restrict__ ev,
    int cap_evt, int cap_cand, uint64_t* __restrict__ best, int32_t* __restrict__ used,
    int8_t* __restrict__ evs, semipar_event* __restrict__ log, int64_t log_cap,
    const uint64_t* __restrict__ blkred, int nblk, Ctrl* ctrl, const int32_t* __restrict__ rid,
    int32_t* __restrict__ log_rid, int32_t* __restrict__ lev, double p_ic, uint64_t seed,
    const RegionGeom* __restrict__ geoms, int n_sub, uint64_t* __restrict__ rext,
    RCell* __restrict__ rcell, double rc_h) {
  __shared__ int s_live, s_nloc, s_last;
  __shared__ int s_nacc, s_npass;
  __shared__ uint64_t s_t[RES_LDS_EVT];
  __shared__ int32_t s_list[RES_LDS_EVT];
  __shared__ int16_t s_la[RES_LDS_EVT], s_lb[RES_LDS_EVT];
  __shared__ int8_t s_evs[RES_LDS_EVT];
  __shared__ int32_t s_hkey[RES_HASH];
  __shared__ uint32_t s_best[RES_HASH];
  __shared__ uint64_t s_min[RESOLVE_NT / 64], s_max[RESOLVE_NT / 64], s_adv[RESOLVE_NT / 64];
  if (ctrl->done) return;
  const int t = threadIdx.x;
  const int ngrp = (int)gridDim.x, grp = (int)blockIdx.x;
  const int ncand = ctrl->n_cand;
  const int ne = ctrl->n_evt;
  int defer = 0;
  if (ncand > cap_cand) defer |= 1;
  if (ne > cap_evt) defer |= 2;
  if (ctrl->log_n + (int64_t)ne > log_cap) defer |= 4;
  const int32_t step_stamp = ctrl->step + 1;
  const uint32_t base = (uint32_t)ctrl->stamp;
  const int32_t n_step = ctrl->step;
  const int64_t log0 = ctrl->log_n;
  // the event's group: its sub-region modulo the workgroups
  auto mine = [&](int e) { return ngrp == 1 || rid[ev[e].sa] % ngrp == grp; };
  if (t == 0) {
    s_nloc = 0;
    s_nacc = 0;
    s_npass = 0;
  }
  __syncthreads();
  uint32_t iter = 0;
  if (!defer && ne > 0) {
    // this group's events (any order: the matching depends on the keys only)
    for (int e = t; e < ne; e += RESOLVE_NT)
      if (mine(e)) {
        const int i = atomicAdd(&s_nloc, 1);
        if (i < RES_LDS_EVT) s_list[i] = e;
      }
    __syncthreads();
    const int nloc = s_nloc;
    const bool in_lds = nloc <= RES_LDS_EVT;
    if (in_lds) {
      for (int i = t; i < RES_HASH; i += RESOLVE_NT) {
        s_hkey[i] = -1;
        s_best[i] = 0;
      }
      __syncthreads();
      // event states: 1 in the matching, 3 passes through (2 accepted, 0 blocked)
      for (int i = t; i < nloc; i += RESOLVE_NT) {
        const EvCand& c = ev[s_list[i]];
        s_evs[i] = (p_ic >= 1.0 || crossing_draw(seed, n_step, c.ida, c.idb) < p_ic) ? 1 : 3;
        s_t[i] = order_bits(c.t);
        s_la[i] = (int16_t)lslot(s_hkey, c.sa);
        s_lb[i] = (int16_t)lslot(s_hkey, c.sb);
      }
      __syncthreads();
      for (;;) {
        const uint32_t tag0 = (iter + 1) << 12;
        for (int i = t; i < nloc; i += RESOLVE_NT)
          if (s_evs[i] == 1) {
            lpropose(s_best, s_la[i], tag0 | (uint32_t)i, i, s_t, s_list, ev);
            lpropose(s_best, s_lb[i], tag0 | (uint32_t)i, i, s_t, s_list, ev);
          }
        __syncthreads();
        // an event holding both its slots is accepted and takes them; an event whose
        // slot holds another tag cannot hold it, so the two checks do not interfere
        for (int i = t; i < nloc; i += RESOLVE_NT)
          if (s_evs[i] == 1) {
            const uint32_t tag = tag0 | (uint32_t)i;
            const int la = s_la[i], lb = s_lb[i];
            if (s_best[la] == tag && s_best[lb] == tag) {
              s_evs[i] = 2;
              s_best[la] = RES_USED;
              s_best[lb] = RES_USED;
            }
          }
        if (t == 0) s_live = 0;
        __syncthreads();
        int live = 0;
        for (int i = t; i < nloc; i += RESOLVE_NT)
          if (s_evs[i] == 1) {
            if (s_best[s_la[i]] == RES_USED || s_best[s_lb[i]] == RES_USED)
              s_evs[i] = 0;
            else
              live++;
          }
        if (live) atomicAdd(&s_live, live);
        __syncthreads();
        const int remaining = s_live;
        __syncthreads();
        ++iter;
        if (remaining == 0) break;
      }
    } else {
      // more events than the LDS holds: the same rounds on per-slot tags in memory
      for (int e = t; e < ne; e += RESOLVE_NT)
        if (mine(e)) {
          const EvCand& c = ev[e];
          evs[e] = (p_ic >= 1.0 || crossing_draw(seed, n_step, c.ida, c.idb) < p_ic) ? 1 : 3;
        }
      __syncthreads();
      for (;;) {
        const uint32_t stp = base + 1 + iter;
        for (int e = t; e < ne; e += RESOLVE_NT)
          if (mine(e) && evs[e] == 1) {
            propose(best, ev[e].sa, stp, e, ev);
            propose(best, ev[e].sb, stp, e, ev);
          }
        __syncthreads();
        const uint64_t tag0 = (uint64_t)stp << 32;
        for (int e = t; e < ne; e += RESOLVE_NT)
          if (mine(e) && evs[e] == 1) {
            const uint64_t tag = tag0 | (uint32_t)e;
            if (aload64(&best[ev[e].sa]) == tag && aload64(&best[ev[e].sb]) == tag) {
              evs[e] = 2;
              astore32(&used[ev[e].sa], step_stamp);
              astore32(&used[ev[e].sb], step_stamp);
            }
          }
        if (t == 0) s_live = 0;
        __syncthreads();
        int live = 0;
        for (int e = t; e < ne; e += RESOLVE_NT)
          if (mine(e) && evs[e] == 1) {
            if (aload32(&used[ev[e].sa]) == step_stamp || aload32(&used[ev[e].sb]) == step_stamp)
              evs[e] = 0;
            else
              live++;
          }
        if (live) atomicAdd(&s_live, live);
        __syncthreads();
        const int remaining = s_live;
        __syncthreads();
        ++iter;
        if (remaining == 0) break;
      }
    }
    // partner exchange (accepted events touch disjoint elements) and log; places in the
    // log are reserved once per wave (the log is put in listing order when read)
    const int nit = in_lds ? nloc : ne;
    const int span = (nit + RESOLVE_NT - 1) / RESOLVE_NT * RESOLVE_NT;  // whole waves
    for (int i = t; i < span; i += RESOLVE_NT) {
      int e = -1;
      int8_t es = 0;
      if (i < nit) {
        if (in_lds) {
          e = s_list[i];
          es = s_evs[i];
        } else if (mine(i)) {
          e = i;
          es = evs[i];
        }
      }
      const bool logged = es == 2 || es == 3;
      const int li = wave_reserve(&ctrl->res_nlog, logged);
      if (!logged) continue;
      const int a = ev[e].sa, b = ev[e].sb;
      if (es == 2) {
        const int ja = nxt[a], jb = nxt[b];
        nxt[a] = jb;
        nxt[b] = ja;
        prv[jb] = a;
        prv[ja] = b;
        atomicAdd(&s_nacc, 1);
      } else {
        atomicAdd(&s_npass, 1);
      }
      semipar_event o;
      o.step = n_step;
      o.kind = es == 2 ? 0 : 1;
      o.id_a = ev[e].ida;
      o.id_b = ev[e].idb;
      o.t_star = ev[e].t;
      o.x_star[0] = ev[e].x;
      o.x_star[1] = ev[e].y;
      o.x_star[2] = ev[e].z;
      log[log0 + li] = o;
      if (log_rid) log_rid[log0 + li] = rid[a];
      lev[a] = n_step;
      lev[b] = n_step;
    }
    __syncthreads();
    if (t == 0) {
      if (s_nacc) atomicAdd(&ctrl->res_nacc, s_nacc);
      if (s_npass) atomicAdd(&ctrl->res_npass, s_npass);
      atomicMax(&ctrl->res_iter, (int32_t)iter);
    }
  }
  // the last workgroup to get here does the step's bookkeeping (every other workgroup
  // has read the control block and written its results by then)
  __syncthreads();
  if (t == 0) {
    __threadfence();
    s_last = atomicAdd(&ctrl->res_done, 1) == ngrp - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (defer) {
    if (t == 0) {
      ctrl->defer = defer;
      ctrl->done = 1;
      ctrl->n_cand = 0;
      ctrl->n_evt = 0;
      ctrl->n_large = 0;
      ctrl->tmin_key = KEY_MAX;
      ctrl->res_done = 0;
    }
    return;
  }
  // smallest t of the slice written by this step's k_evolve, largest element extent
  uint64_t mk = KEY_MAX, xk = 0, ak = 0;
  for (int b = t; b < nblk; b += RESOLVE_NT) {
    mk = blkred[4 * b] < mk ? blkred[4 * b] : mk;
    xk = blkred[4 * b + 1] > xk ? blkred[4 * b + 1] : xk;
    ak += blkred[4 * b + 2];
  }
  mk = wave_min_u64(mk);
  xk = wave_max_u64(xk);
  for (int o = 32; o > 0; o >>= 1) ak += __shfl_xor(ak, o, 64);
  if ((t & 63) == 0) {
    s_min[t >> 6] = mk;
    s_max[t >> 6] = xk;
    s_adv[t >> 6] = ak;
  }
  __syncthreads();
  if (t == 0) {
    uint64_t m = s_min[0], x = s_max[0], nadv = s_adv[0];
    for (int w = 1; w < RESOLVE_NT / 64; ++w) {
      m = s_min[w] < m ? s_min[w] : m;
      x = s_max[w] > x ? s_max[w] : x;
      nadv += s_adv[w];
    }
    const int32_t nlog = aload32(&ctrl->res_nlog);
    const int32_t nacc = aload32(&ctrl->res_nacc);
    const int32_t npass = aload32(&ctrl->res_npass);
    const int32_t rounds = aload32(&ctrl->res_iter);
    if (!ctrl->cells.fixed && x != 0)
      ctrl->cells = choose_cells(ctrl->box, ctrl->grow * from_key(x), ctrl->tol);
    ctrl->log_n += nlog;
    ctrl->acc_total += nacc;
    ctrl->pass_total += npass;
    ctrl->conf_total += ne;
    ctrl->cand_total += ncand;
    ctrl->last_cand = ncand;
    ctrl->large_total += ctrl->n_large;
    ctrl->n_cand = 0;
    ctrl->n_evt = 0;
    ctrl->n_large = 0;
    ctrl->res_nlog = 0;
    ctrl->res_nacc = 0;
    ctrl->res_npass = 0;
    ctrl->res_iter = 0;
    ctrl->res_done = 0;
    ctrl->stamp = (int32_t)(base + (uint32_t)rounds);
    ctrl->step += 1;
    ctrl->steps_taken += 1;
    ctrl->point_steps += (int64_t)nadv;
    const double tmin = nadv ? from_key(m) : 0.0;
    ctrl->done = (ctrl->step >= ctrl->step_limit || (nadv == 0 && ctrl->step > ctrl->start_last) ||
                  tmin >= ctrl->t_end)
                     ? 1
                     : 0;
  }
  // a batch: every sub-region's grid for the next step (the events' LDS is free now)
  if (rcell) {
    __syncthreads();
    if (!(rc_h <= 0.0 && ctrl->done))
      rcells_update(geoms, n_sub, rext, rcell, rc_h, ctrl, s_t);
  }
}

// ---------------------------------------------------------------------------------
// persistent evolution of small regions
// ---------------------------------------------------------------------------------
// A batch of small bounded regions in one launch: each workgroup takes the next
// sub-region from a device counter and evolves it through all of its steps without
// leaving the kernel (workgroup barriers between the phases of a step), then takes the
// next. Per step, the same arithmetic as the step kernels: decisions and diamond tops,
// the elements of the band, every pair of elements of the region tested with the exact
// FP64 4-D box test that the confirmation applies (which the screen only pre-filters),
// the four triangle pairs, and the greedy matching in (t*, id_a, id_b) order, taken one
// event after another. So each region ends exactly as a run of it alone. A step with
// more crossings than the workgroup holds stops the launch (error bit 64): the caller
// runs the batch again from its surfaces on the step kernels.
constexpr int PB_NT = 256;    // threads of a workgroup
constexpr int PB_MAXP = SEMIPAR_PERSISTENT_MAX;  // most points of a region evolved this way
constexpr int PB_EVT = SEMIPAR_PERSISTENT_EVENTS;  // crossings of one step held in LDS
constexpr int PB_GRID = 1024; // most workgroups

struct PbEv {
  double t, x, y, z;
  int64_t ida, idb;
  int32_t sa, sb;
};

template <bool FRW>
__global__ __launch_bounds__(PB_NT) void k_region_block(
    Slices X, int32_t* __restrict__ nxt, int32_t* __restrict__ prv,
    const int64_t* __restrict__ id, int32_t* __restrict__ fstep, int32_t* __restrict__ face,
    semipar_point_rec* __restrict__ frz, int32_t* __restrict__ lev,
    const RegionGeom* __restrict__ geoms, const int64_t* __restrict__ sub_off, int n_sub,
    int32_t* __restrict__ work_head, sp::Period P, double hcoef, int32_t step0,
    int32_t step_limit, double p_ic, uint64_t seed, semipar_event* __restrict__ log,
    int32_t* __restrict__ log_rid, int64_t log_cap, Ctrl* ctrl) {
  __shared__ double s_lo[PB_MAXP][4], s_hi[PB_MAXP][4];
  __shared__ double s_anc[PB_MAXP][3];
  __shared__ int64_t s_id[PB_MAXP];
  __shared__ uint8_t s_adv[PB_MAXP], s_val[PB_MAXP], s_used[PB_MAXP];
  __shared__ PbEv s_ev[PB_EVT];
  __shared__ int s_q, s_nadv, s_nev, s_ncand, s_abort;
  __shared__ int s_ord[PB_EVT];
  __shared__ int8_t s_kind[PB_EVT];
  const int t = threadIdx.x;
  for (;;) {
    if (t == 0) s_q = atomicAdd(work_head, 1);
    __syncthreads();
    const int q = s_q;
    if (q >= n_sub) return;
    const int64_t off = sub_off[q];
    const int n = (int)(sub_off[q + 1] - off);
    const RegionGeom G = geoms[q];
    int64_t psteps = 0, ncand = 0, nconf = 0, nacc = 0, npass = 0;
    int32_t s = step0;
    bool aborted = false;
    while (n > 0 && s < step_limit) {
      const int ic = s % 3, ip = (s + 2) % 3, in = (s + 1) % 3;
      if (t == 0) {
        s_nadv = 0;
        s_nev = 0;
        s_ncand = 0;
        s_abort = ctrl->err & 64;  // another workgroup gave up: so does this one
      }
      __syncthreads();
      if (s_abort) {
        aborted = true;
        break;
      }
      // decisions and tops (as k_evolve for a bounded region)
      int my_adv = 0;
      for (int i = t; i < n; i += PB_NT) {
        const int k = (int)off + i;
        bool adv = false;
        if (fstep[k] == FS_ACTIVE) {
          const int j = nxt[k];
          int f = -1;
          bool with_r = false;
          V4 B{}, R{};
          if (j >= 0) {
            B = ld(X, ip, j);
            R = ld(X, ic, j);
          }
          if (j < 0) {
            f = -1;
          } else if (fstep[j] < s) {
            f = face[j];
          } else {
            f = exit_face(G, B);
            if (f < 0) adv = true;
            with_r = true;
          }
          if (!adv) {
            write_frozen(frz, X, ic, ip, k, j, with_r, f, s, prv, id);
            face[k] = f;
            fstep[k] = s;
          } else {
            const V4 L = ld(X, ic, k);
            st(X, in, k, sp::top<FRW>(L, R, B, P, hcoef));
            ++my_adv;
          }
        }
        s_adv[i] = adv ? 1 : 0;
      }
      if (my_adv) atomicAdd(&s_nadv, my_adv);
      __syncthreads();
      const int nadv = s_nadv;
      if (nadv == 0) {  // every point has stopped: this step counts as taken, as on the
        ++s;            // step kernels
        break;
      }
      psteps += nadv;
      // the elements of band s: k and next[k] both advanced
      for (int i = t; i < n; i += PB_NT) {
        uint8_t v = 0;
        if (s_adv[i]) {
          const int k = (int)off + i;
          const int j = nxt[k];
          if (s_adv[j - (int)off]) {
            const Elem e = sp::make_elem(ld(X, ic, k), ld(X, ic, j), ld(X, in, k), ld(X, in, j), P);
            const Box4 b = sp::elem_box(e);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              s_lo[i][c] = b.lo[c];
              s_hi[i][c] = b.hi[c];
            }
            s_anc[i][0] = e.v[0].x;
            s_anc[i][1] = e.v[0].y;
            s_anc[i][2] = e.v[0].z;
            v = 1;
          }
        }
        s_val[i] = v;
        s_used[i] = 0;
        if (s == step0) s_id[i] = id[(int)off + i];
      }
      __syncthreads();
      // every pair of elements of the region: exact box overlap, then the triangle pairs
      int my_cand = 0;
      for (int i = t; i < n; i += PB_NT) {
        if (!s_val[i]) continue;
        const int k = (int)off + i;
        const int nk = nxt[k] - (int)off, pk = prv[k] - (int)off;
        const int64_t idi = s_id[i];
        for (int m = i + 1; m < n; ++m) {
          if (!s_val[m] || m == nk || m == pk) continue;
          // a = the element of the point with the smaller id (the order the
          // confirmation uses)
          int a = i, b = m;
          if (s_id[m] < idi) {
            a = m;
            b = i;
          }
          double S[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) S[c] = P.box * P.nearest(s_anc[b][c] - s_anc[a][c]);
          bool ov = true;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            ov = ov && (s_lo[a][c] <= s_hi[b][c] - S[c]) && (s_lo[b][c] - S[c] <= s_hi[a][c]);
          ov = ov && (s_lo[a][3] <= s_hi[b][3]) && (s_lo[b][3] <= s_hi[a][3]);
          if (!ov) continue;
          ++my_cand;
          const int ga = (int)off + a, gb = (int)off + b;
          const Elem ea = load_elem(X, ic, in, ga, nxt[ga], P);
          Elem eb = load_elem(X, ic, in, gb, nxt[gb], P);
          for (int v = 0; v < 4; ++v) {
            eb.v[v].x = eb.v[v].x - S[0];
            eb.v[v].y = eb.v[v].y - S[1];
            eb.v[v].z = eb.v[v].z - S[2];
          }
          bool found = false;
          double bt = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
          for (int ipq = 0; ipq < 4; ++ipq) {
            const int ipp = ipq >> 1, iq = ipq & 1;
            double tt, xx, yy, zz;
            if (sp::tri_tri(ipp ? ea.v[2] : ea.v[0], ea.v[1], ipp ? ea.v[3] : ea.v[2],
                            iq ? eb.v[2] : eb.v[0], eb.v[1], iq ? eb.v[3] : eb.v[2], tt, xx, yy,
                            zz)) {
              if (!found || tt < bt) {
                found = true;
                bt = tt;
                bx = xx;
                by = yy;
                bz = zz;
              }
            }
          }
          if (!found) continue;
          const int e = atomicAdd(&s_nev, 1);
          if (e < PB_EVT) {
            PbEv c;
            c.t = bt;
            c.x = bx;
            c.y = by;
            c.z = bz;
            c.ida = id[ga];
            c.idb = id[gb];
            c.sa = ga;
            c.sb = gb;
            s_ev[e] = c;
          }
        }
      }
      if (my_cand) atomicAdd(&s_ncand, my_cand);
      __syncthreads();
      const int ne = s_nev;
      if (ne > PB_EVT) {
        if (t == 0) atomicOr(&ctrl->err, 64);
        aborted = true;
        break;
      }
      ncand += s_ncand;
      nconf += ne;
      // the greedy matching in (t*, id_a, id_b) order, one event after another, after
      // each crossing's draw (p < 1: a draw >= p passes through, claims nothing)
      if (t == 0 && ne > 0) {
        for (int e = 0; e < ne; ++e) s_ord[e] = e;
        for (int e = 1; e < ne; ++e) {  // insertion sort by key
          const int x = s_ord[e];
          int f = e - 1;
          while (f >= 0) {
            const PbEv& A = s_ev[s_ord[f]];
            const PbEv& Bv = s_ev[x];
            const bool gt = A.t > Bv.t || (A.t == Bv.t && (A.ida > Bv.ida ||
                                                            (A.ida == Bv.ida && A.idb > Bv.idb)));
            if (!gt) break;
            s_ord[f + 1] = s_ord[f];
            --f;
          }
          s_ord[f + 1] = x;
        }
        int nlog = 0;
        for (int o = 0; o < ne; ++o) {
          const PbEv& c = s_ev[s_ord[o]];
          int8_t kind = -1;
          if (!(p_ic >= 1.0 || crossing_draw(seed, s, c.ida, c.idb) < p_ic)) {
            kind = 1;
          } else if (!s_used[c.sa - (int)off] && !s_used[c.sb - (int)off]) {
            kind = 0;
            s_used[c.sa - (int)off] = 1;
            s_used[c.sb - (int)off] = 1;
          }
          s_kind[o] = kind;
          if (kind >= 0) ++nlog;
        }
        const int64_t base = atomicAdd((unsigned long long*)&ctrl->log_n, (unsigned long long)nlog);
        if (base + nlog > log_cap) {
          atomicOr(&ctrl->err, 64);
          s_abort = 1;
        } else {
          int li = 0;
          for (int o = 0; o < ne; ++o) {
            if (s_kind[o] < 0) continue;
            const PbEv& c = s_ev[s_ord[o]];
            if (s_kind[o] == 0) {
              const int ja = nxt[c.sa], jb = nxt[c.sb];
              nxt[c.sa] = jb;
              nxt[c.sb] = ja;
              prv[jb] = c.sa;
              prv[ja] = c.sb;
              ++nacc;
            } else {
              ++npass;
            }
            semipar_event ev;
            ev.step = s;
            ev.kind = s_kind[o];
            ev.id_a = c.ida;
            ev.id_b = c.idb;
            ev.t_star = c.t;
            ev.x_star[0] = c.x;
            ev.x_star[1] = c.y;
            ev.x_star[2] = c.z;
            log[base + li] = ev;
            if (log_rid) log_rid[base + li] = q;
            lev[c.sa] = s;
            lev[c.sb] = s;
            ++li;
          }
        }
      }
      __syncthreads();
      if (s_abort) {
        aborted = true;
        break;
      }
      ++s;
    }
    // this region's totals (thread 0 holds the matching's counts)
    if (t == 0 && !aborted) {
      atomicAdd((unsigned long long*)&ctrl->point_steps, (unsigned long long)psteps);
      atomicAdd((unsigned long long*)&ctrl->cand_total, (unsigned long long)ncand);
      atomicAdd((unsigned long long*)&ctrl->conf_total, (unsigned long long)nconf);
      atomicAdd((unsigned long long*)&ctrl->acc_total, (unsigned long long)nacc);
      atomicAdd((unsigned long long*)&ctrl->pass_total, (unsigned long long)npass);
      atomicMax(&ctrl->pb_step, s);  // the furthest slice any region reached
    }
    __syncthreads();
  }
}

// Start of an evolve call: per block, the smallest t on the current slice and the number
// of points still advancing (all points of a whole-volume region).
__global__ __launch_bounds__(NT) void k_begin_min(Slices X, int n, const int32_t* fstep,
                                                  uint64_t* __restrict__ blkred, Ctrl* ctrl) {
  const int s = ctrl->step;
  const int k = blockIdx.x * NT + threadIdx.x;
  uint64_t key = KEY_MAX;
  uint32_t act = 0;
  if (k < n && (!fstep || fstep[k] == FS_ACTIVE)) {
    key = order_key(X.p[s % 3][k].w);
    act = 1;
  }
  __shared__ uint64_t wmin[NT / 64];
  __shared__ uint32_t wact[NT / 64];
  key = wave_min_u64(key);
  for (int o = 32; o > 0; o >>= 1) act += __shfl_xor(act, o, 64);
  if ((threadIdx.x & 63) == 0) {
    wmin[threadIdx.x >> 6] = key;
    wact[threadIdx.x >> 6] = act;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t m = wmin[0], a = wact[0];
    for (int w = 1; w < NT / 64; ++w) {
      m = wmin[w] < m ? wmin[w] : m;
      a += wact[w];
    }
    blkred[4 * blockIdx.x] = m;
    blkred[4 * blockIdx.x + 1] = 0;
    blkred[4 * blockIdx.x + 2] = a;
  }
}

__global__ __launch_bounds__(1024) void k_begin_set(Ctrl* ctrl, int32_t step_limit, double t_end,
                                                    const uint64_t* __restrict__ blkred, int nblk,
                                                    Cells cells, int set_cells, double grow) {
  __shared__ uint64_t s_min[16], s_act[16];
  const int t = threadIdx.x;
  uint64_t mk = KEY_MAX, ak = 0;
  for (int b = t; b < nblk; b += 1024) {
    mk = blkred[4 * b] < mk ? blkred[4 * b] : mk;
    ak += blkred[4 * b + 2];
  }
  mk = wave_min_u64(mk);
  for (int o = 32; o > 0; o >>= 1) ak += __shfl_xor(ak, o, 64);
  if ((t & 63) == 0) {
    s_min[t >> 6] = mk;
    s_act[t >> 6] = ak;
  }
  __syncthreads();
  if (t != 0) return;
  uint64_t m = s_min[0], a = s_act[0];
  for (int w = 1; w < 16; ++w) {
    m = s_min[w] < m ? s_min[w] : m;
    a += s_act[w];
  }
  if (set_cells) ctrl->cells = cells;
  ctrl->grow = grow;
  ctrl->step_limit = step_limit;
  ctrl->t_end = t_end;
  ctrl->defer = 0;
  ctrl->n_cand = 0;
  ctrl->n_evt = 0;
  ctrl->n_large = 0;
  const double tmin = a ? from_key(m) : 0.0;
  ctrl->done = (a == 0 || ctrl->step >= step_limit || tmin >= t_end) ? 1 : 0;
}

// ---- loop record and removal ---------------------------------------------------------
// Section "Semi-parallel cosmic string simulation": a loop that will not meet anything
// again is logged and taken out. Chains of still-advancing points are labelled by list
// ranking (pointer doubling): after R rounds with 2^R >= n, lab[k] is the smallest slot
// of k's chain when the chain closes on itself through advancing points, else LAB_OPEN
// (following next from k reaches a point whose right neighbour is missing or stopped).
// Links form a partial permutation (init checks the next/prev pairing and a partner
// exchange keeps it), so every chain is a cycle or a path.
constexpr int32_t LAB_OPEN = -1;
constexpr int32_t LAB_NONE = -2;  // the point no longer advances

// Nearest periodic image of a spatial difference, as d - L rint(d / L).
__device__ __forceinline__ double wrap_box(double d, double box) {
  return d - box * rint(d / box);
}

__global__ __launch_bounds__(NT) void k_loop_init(int n, const int32_t* __restrict__ nxt,
                                                  const int32_t* __restrict__ fstep,
                                                  int32_t* __restrict__ lab,
                                                  int32_t* __restrict__ ptr,
                                                  int32_t* __restrict__ lcnt,
                                                  int32_t* __restrict__ levm,
                                                  int32_t* __restrict__ lbad) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n) return;
  int32_t l = LAB_NONE, q = k;
  if (fstep[k] == FS_ACTIVE) {
    const int j = nxt[k];
    const bool end = j < 0 || fstep[j] != FS_ACTIVE;
    l = end ? LAB_OPEN : k;
    q = end ? k : j;  // a chain's end points to itself
  }
  lab[k] = l;
  ptr[k] = q;
  lcnt[k] = 0;
  levm[k] = INT32_MIN;
  lbad[k] = 0;
}

// One doubling round: lab covers 2^(r+1) successors, ptr jumps 2^(r+1) links.
__global__ __launch_bounds__(NT) void k_loop_jump(int n, const int32_t* __restrict__ lab_in,
                                                  const int32_t* __restrict__ ptr_in,
                                                  int32_t* __restrict__ lab_out,
                                                  int32_t* __restrict__ ptr_out) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n) return;
  const int32_t l = lab_in[k];
  const int q = ptr_in[k];
  if (l == LAB_NONE) {
    lab_out[k] = LAB_NONE;
    ptr_out[k] = q;
    return;
  }
  const int32_t lq = lab_in[q];
  lab_out[k] = lq < l ? lq : l;
  ptr_out[k] = ptr_in[q];
}

// Per closed chain (indexed by its lowest slot): point count, latest event step, and
// whether some point lies a quarter box or more from the lowest slot's point (per axis,
// nearest image). One atomic per wave where the wave holds one chain.
__global__ __launch_bounds__(NT) void k_loop_gather(int n, int s, Slices X,
                                                    const int32_t* __restrict__ lab,
                                                    const int32_t* __restrict__ lev, double box,
                                                    int32_t* __restrict__ lcnt,
                                                    int32_t* __restrict__ levm,
                                                    int32_t* __restrict__ lbad) {
  const int k = blockIdx.x * NT + threadIdx.x;
  const int32_t q = k < n ? lab[k] : LAB_NONE;
  const bool live = q >= 0;
  int32_t e = INT32_MIN, bad = 0;
  if (live) {
    const int ic = s % 3;
    const V4 a = ld(X, ic, k), b = ld(X, ic, q);
    const double lim = 0.25 * box;
    bad = (fabs(wrap_box(a.x - b.x, box)) < lim && fabs(wrap_box(a.y - b.y, box)) < lim &&
           fabs(wrap_box(a.z - b.z, box)) < lim)
              ? 0
              : 1;
    e = lev[k];
  }
  if (wave_uniform(q, live)) {
    int32_t c = live ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) {
      c += __shfl_xor(c, o, 64);
      const int32_t e2 = __shfl_xor(e, o, 64);
      e = e2 > e ? e2 : e;
      bad |= __shfl_xor(bad, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&lcnt[q], c);
      atomicMax(&levm[q], e);
      if (bad) atomicOr(&lbad[q], 1);
    }
  } else if (live) {
    atomicAdd(&lcnt[q], 1);
    atomicMax(&levm[q], e);
    if (bad) atomicOr(&lbad[q], 1);
  }
}

// Decision per closed chain of L points at the start of step s: removed when compact
// and no event in steps s - L .. s - 1 (s - latest > L). Accepted chains get a loop
// index (completion order); ctr[0] counts loops, ctr[1] their points.
__global__ __launch_bounds__(NT) void k_loop_decide(int n, int s, const int32_t* __restrict__ lab,
                                                    const int32_t* __restrict__ lcnt,
                                                    const int32_t* __restrict__ levm,
                                                    const int32_t* __restrict__ lbad,
                                                    int32_t* __restrict__ lidx,
                                                    int32_t* __restrict__ lrep,
                                                    int32_t* __restrict__ ctr) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n || lab[k] != k) return;
  const int32_t L = lcnt[k];
  int32_t li = -1;
  if (!lbad[k] && (int64_t)s - (int64_t)levm[k] > (int64_t)L) {
    li = atomicAdd(&ctr[0], 1);
    atomicAdd(&ctr[1], L);
    lrep[li] = k;
  }
  lidx[k] = li;
}

// Points of accepted loops: energy and centre sums, then the point stops at slice s
// (record flagged REMOVED, no owning face, no element from now on).
__global__ __launch_bounds__(NT) void k_loop_apply(int n, int s, Slices X,
                                                   const int32_t* __restrict__ lab,
                                                   const int32_t* __restrict__ lidx,
                                                   const int32_t* __restrict__ nxt,
                                                   const int32_t* __restrict__ prv,
                                                   const int64_t* __restrict__ id, double box,
                                                   double* __restrict__ lacc,
                                                   semipar_point_rec* __restrict__ frz,
                                                   int32_t* __restrict__ fstep,
                                                   int32_t* __restrict__ face,
                                                   int32_t* __restrict__ ecell) {
  const int k = blockIdx.x * NT + threadIdx.x;
  const int32_t q = k < n ? lab[k] : LAB_NONE;
  const int32_t li = q >= 0 ? lidx[q] : -1;
  const bool live = li >= 0;
  double e = 0.0, c[3] = {0.0, 0.0, 0.0};
  if (live) {
    const int ic = s % 3, ip = (s + 2) % 3;
    const int j = nxt[k];
    const V4 a = ld(X, ic, k), aj = ld(X, ic, j), pj = ld(X, ip, j), r0 = ld(X, ic, q);
    const double d0 = wrap_box(a.x - pj.x, box), d1 = wrap_box(a.y - pj.y, box),
                 d2 = wrap_box(a.z - pj.z, box);
    const double f0 = aj.x - pj.x, f1 = aj.y - pj.y, f2 = aj.z - pj.z;
    e = sqrt(d0 * d0 + d1 * d1 + d2 * d2) + sqrt(f0 * f0 + f1 * f1 + f2 * f2);
    c[0] = wrap_box(a.x - r0.x, box);
    c[1] = wrap_box(a.y - r0.y, box);
    c[2] = wrap_box(a.z - r0.z, box);
    semipar_point_rec r;
    r.id = id[k];
    const int pk = prv[k];
    r.next_id = id[j];
    r.prev_id = pk >= 0 ? id[pk] : -1;
    r.step = s;
    r.flags = SEMIPAR_FLAG_REMOVED;
    const V4 b = ld(X, ip, k);
    r.x[0] = a.x; r.x[1] = a.y; r.x[2] = a.z; r.x[3] = a.t;
    r.x_prev[0] = b.x; r.x_prev[1] = b.y; r.x_prev[2] = b.z; r.x_prev[3] = b.t;
    for (int i = 0; i < 4; ++i) {
      r.r[i] = 0.0;
      r.r_prev[i] = 0.0;
    }
    frz[k] = r;
    fstep[k] = s;
    face[k] = -1;
    if (ecell) ecell[k] = NO_ELEM;
  }
  if (wave_uniform(li, live)) {
    for (int o = 32; o > 0; o >>= 1) {
      e += __shfl_xor(e, o, 64);
      for (int i = 0; i < 3; ++i) c[i] += __shfl_xor(c[i], o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&lacc[4 * li], e);
      for (int i = 0; i < 3; ++i) atomicAdd(&lacc[4 * li + 1 + i], c[i]);
    }
  } else if (live) {
    atomicAdd(&lacc[4 * li], e);
    for (int i = 0; i < 3; ++i) atomicAdd(&lacc[4 * li + 1 + i], c[i]);
  }
}

// Loop records: centre = lowest slot's point + mean nearest-image displacement.
__global__ __launch_bounds__(NT) void k_loop_final(int nl, int s, Slices X,
                                                   const int32_t* __restrict__ lrep,
                                                   const int32_t* __restrict__ lcnt,
                                                   const int64_t* __restrict__ id,
                                                   const double* __restrict__ lacc,
                                                   const int32_t* __restrict__ rid,
                                                   semipar_loop* __restrict__ out,
                                                   int32_t* __restrict__ out_rid) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= nl) return;
  const int q = lrep[i];
  const int32_t L = lcnt[q];
  const V4 r0 = ld(X, s % 3, q);
  semipar_loop o;
  o.step = s;
  o.n_points = L;
  o.rep_id = id[q];
  o.energy = lacc[4 * i];
  o.centre[0] = r0.x + lacc[4 * i + 1] / (double)L;
  o.centre[1] = r0.y + lacc[4 * i + 2] / (double)L;
  o.centre[2] = r0.z + lacc[4 * i + 3] / (double)L;
  out[i] = o;
  if (out_rid) out_rid[i] = rid ? rid[q] : 0;
}

// Local grids of the sub-regions of a batch for the next step (one workgroup). h_set > 0:
// every region gets cells of edge >= h_set (start of a call, or a fixed cell size);
// otherwise each region's cells follow its own largest element of the step just taken
// (grow x extent; regions without elements keep their grid). Bucket bases are the
// running sum of the regions' cell counts. The extents are reset for the next step.
// The grids of the first step of an evolve call (the per-step update runs in the last
// workgroup of k_resolve).
__global__ __launch_bounds__(1024) void k_rcells(const RegionGeom* __restrict__ geoms, int n_sub,
                                                 uint64_t* __restrict__ rext,
                                                 RCell* __restrict__ rc, double h_set,
                                                 const Ctrl* ctrl) {
  if (h_set <= 0.0 && ctrl->done) return;
  __shared__ uint64_t s_sum[1024];
  rcells_update(geoms, n_sub, rext, rc, h_set, ctrl, s_sum);
}

// ---------------------------------------------------------------------------------
// init / emit kernels
// ---------------------------------------------------------------------------------
constexpr int64_t ID_EMPTY = INT64_MIN;

__device__ __forceinline__ uint32_t id_hash(int64_t id, uint32_t mask) {
  uint64_t z = (uint64_t)id + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (uint32_t)z & mask;
}

__global__ __launch_bounds__(NT) void k_init_insert(const semipar_point_rec* __restrict__ rec,
                                                    int n, int64_t* __restrict__ hkey,
                                                    int32_t* __restrict__ hval, uint32_t hmask,
                                                    Ctrl* ctrl) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n) return;
  const int64_t id = rec[k].id;
  if (id == ID_EMPTY) {
    atomicOr(&ctrl->err, 1);
    return;
  }
  uint32_t h = id_hash(id, hmask);
  for (uint32_t probe = 0; probe <= hmask; ++probe) {
    const unsigned long long prev = atomicCAS((unsigned long long*)&hkey[h],
                                              (unsigned long long)ID_EMPTY, (unsigned long long)id);
    if ((int64_t)prev == ID_EMPTY) {
      hval[h] = k;
      return;
    }
    if ((int64_t)prev == id) {
      atomicOr(&ctrl->err, 2);  // duplicate id
      return;
    }
    h = (h + 1) & hmask;
  }
  atomicOr(&ctrl->err, 4);
}

// Sub-region of every slot of a batch from the first slot of each sub-region (off has
// n_sub + 1 non-decreasing entries, off[n_sub] = n): the last q with off[q] <= k.
__global__ __launch_bounds__(NT) void k_fill_rid(int32_t* __restrict__ rid, int n,
                                                 const int64_t* __restrict__ off, int n_sub) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n) return;
  int lo = 0, hi = n_sub - 1;  // off[lo] <= k < off[hi + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= (int64_t)k) lo = mid;
    else hi = mid - 1;
  }
  rid[k] = lo;
}

__global__ __launch_bounds__(NT) void k_fill_i32(int32_t* p, uint64_t m, int32_t v) {
  const uint64_t i = blockIdx.x * (uint64_t)NT + threadIdx.x;
  if (i < m) p[i] = v;
}

__global__ __launch_bounds__(NT) void k_fill_i64(int64_t* p, uint64_t m, int64_t v) {
  const uint64_t i = blockIdx.x * (uint64_t)NT + threadIdx.x;
  if (i < m) p[i] = v;
}

__device__ __forceinline__ int id_lookup(const int64_t* hkey, const int32_t* hval, uint32_t hmask,
                                         int64_t id) {
  if (id < 0) return -1;
  uint32_t h = id_hash(id, hmask);
  for (uint32_t probe = 0; probe <= hmask; ++probe) {
    const int64_t key = hkey[h];
    if (key == id) return hval[h];
    if (key == ID_EMPTY) return -1;
    h = (h + 1) & hmask;
  }
  return -1;
}

// Links of every point. In a batch (rid set) a link whose target lies in another
// sub-region is cut (-1), exactly as a separate run of the sub-region, which never sees
// the other sub-region's points, leaves it dangling: links never leave a sub-region.
__global__ __launch_bounds__(NT) void k_init_links(const semipar_point_rec* __restrict__ rec, int n,
                                                   const int64_t* __restrict__ hkey,
                                                   const int32_t* __restrict__ hval,
                                                   uint32_t hmask, Slices X, int32_t* nxt,
                                                   int32_t* prv, int64_t* id, int bounded,
                                                   int32_t* fstep, int32_t* face, int32_t* lev,
                                                   const int32_t* __restrict__ rid, Ctrl* ctrl) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n) return;
  const semipar_point_rec r = rec[k];
  const int s = r.step;
  if (s != rec[0].step || s < 1) atomicOr(&ctrl->err, 8);
  int a = id_lookup(hkey, hval, hmask, r.next_id);
  int b = id_lookup(hkey, hval, hmask, r.prev_id);
  if (rid) {
    const int q = rid[k];
    if (a >= 0 && rid[a] != q) a = -1;
    if (b >= 0 && rid[b] != q) b = -1;
  }
  fstep[k] = FS_ACTIVE;
  face[k] = -1;
  lev[k] = s - 1;  // no event yet: as if the last one were before the initial slice
  if (bounded) {
    nxt[k] = a;
    prv[k] = b;
  } else {
    if (a < 0 || b < 0) atomicOr(&ctrl->err, 16);
    nxt[k] = a < 0 ? k : a;
    prv[k] = b < 0 ? k : b;
  }
  id[k] = r.id;
  const int ic = ((s % 3) + 3) % 3, ip = (ic + 2) % 3;
  st(X, ic, k, V4{r.x[0], r.x[1], r.x[2], r.x[3]});
  st(X, ip, k, V4{r.x_prev[0], r.x_prev[1], r.x_prev[2], r.x_prev[3]});
}

// next/prev pairing and an estimate of the element size for the automatic cell.
__global__ __launch_bounds__(NT) void k_init_check(Slices X, int n, const int32_t* nxt,
                                                   const int32_t* prv, sp::Period P, int s,
                                                   Ctrl* ctrl) {
  const int k = blockIdx.x * NT + threadIdx.x;
  uint64_t key = 0;
  if (k < n) {
    const int pk = prv[k];
    if (pk >= 0 && nxt[pk] != k) atomicOr(&ctrl->err, 32);
    const int j = nxt[k];
    if (j >= 0 && prv[j] != k) atomicOr(&ctrl->err, 32);
    const int ic = s % 3, ip = (s + 2) % 3;
    const V4 a = ld(X, ic, k), b = ld(X, ic, j >= 0 ? j : k), c = ld(X, ip, k);
    double e1 = fabs(sp::min_image(b.x - a.x, P));
    e1 = fmax(e1, fabs(sp::min_image(b.y - a.y, P)));
    e1 = fmax(e1, fabs(sp::min_image(b.z - a.z, P)));
    double e2 = fmax(fmax(fabs(a.x - c.x), fabs(a.y - c.y)), fabs(a.z - c.z));
    key = order_key(e1 + e2);
  }
  key = wave_max_u64(key);
  // one atomic per block on the shared estimate
  __shared__ uint64_t wk[NT / 64];
  if ((threadIdx.x & 63) == 0) wk[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t m = wk[0];
    for (int w = 1; w < NT / 64; ++w) m = wk[w] > m ? wk[w] : m;
    atomicMax((unsigned long long*)&ctrl->ext_key, (unsigned long long)m);
  }
}

// Output record of slot k and the surface stream it goes to: a stopped point of a
// bounded region goes to its face (no owning face, or a removed loop: stream 0); a
// point still on the current slice goes to stream 0 (flag ACTIVE in a bounded region).
__device__ __forceinline__ int emit_stream(int k, const int32_t* fstep,
                                           const semipar_point_rec* frz) {
  if (fstep && fstep[k] != FS_ACTIVE) {
    const int f = ((frz[k].flags >> 8) & 0xff) - 1;
    return f >= 0 && f < 4 ? f : 0;
  }
  return 0;
}

__device__ __forceinline__ semipar_point_rec current_record(const Slices& X, int k, int s,
                                                            const int32_t* nxt, const int32_t* prv,
                                                            const int64_t* id, int32_t flags) {
  const int ic = s % 3, ip = (s + 2) % 3;
  semipar_point_rec r;
  r.id = id[k];
  r.next_id = nxt[k] >= 0 ? id[nxt[k]] : -1;
  r.prev_id = prv[k] >= 0 ? id[prv[k]] : -1;
  r.step = s;
  r.flags = flags;
  const V4 a = ld(X, ic, k), b = ld(X, ip, k);
  r.x[0] = a.x;
  r.x[1] = a.y;
  r.x[2] = a.z;
  r.x[3] = a.t;
  r.x_prev[0] = b.x;
  r.x_prev[1] = b.y;
  r.x_prev[2] = b.z;
  r.x_prev[3] = b.t;
  for (int c = 0; c < 4; ++c) {
    r.r[c] = 0.0;
    r.r_prev[c] = 0.0;
  }
  return r;
}

// Per block, the number of records of each of the 4 streams.
// ---- the list of advancing points of a bounded region ----------------------------------
// Rebuilt at the start of every block of steps (count per workgroup, scan, write), so that
// the per-point kernels' waves hold only points that still advanced then; points that
// stop inside the block stay listed and are passed over by their stop step.
// A hand-off batch (start != nullptr) lists only the points that start by the block's last
// step (its step + horizon); later ones are listed by a later block.
__device__ __forceinline__ bool act_listed(int k, int n, const int32_t* __restrict__ fstep,
                                           const int32_t* __restrict__ start, int last) {
  return k < n && fstep[k] == FS_ACTIVE && (!start || start[k] <= last);
}

__global__ __launch_bounds__(NT) void k_act_count(int n, const int32_t* __restrict__ fstep,
                                                  const int32_t* __restrict__ start, int horizon,
                                                  int32_t* __restrict__ blkcnt, const Ctrl* ctrl) {
  if (ctrl->done) return;
  const int k = blockIdx.x * NT + threadIdx.x;
  const uint64_t m = __ballot(act_listed(k, n, fstep, start, ctrl->step + horizon));
  __shared__ int wc[NT / 64];
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < NT / 64; ++w) t += wc[w];
    blkcnt[blockIdx.x] = t;
  }
}

// Exclusive scan of the per-workgroup counts in place (one workgroup); the total is the
// list's length.
__global__ __launch_bounds__(1024) void k_act_scan(int nblk, int32_t* __restrict__ blkcnt,
                                                   Ctrl* ctrl) {
  if (ctrl->done) return;
  __shared__ int sc[1024];
  const int t = threadIdx.x;
  const int per = (nblk + 1023) / 1024;
  const int b0 = t * per, b1 = b0 + per < nblk ? b0 + per : nblk;
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += blkcnt[b];
  sc[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int add = t >= o ? sc[t - o] : 0;
    __syncthreads();
    sc[t] += add;
    __syncthreads();
  }
  int run = sc[t] - sum;
  for (int b = b0; b < b1; ++b) {
    const int c = blkcnt[b];
    blkcnt[b] = run;
    run += c;
  }
  if (t == 1023) ctrl->n_act = sc[1023];
}

__global__ __launch_bounds__(NT) void k_act_write(int n, const int32_t* __restrict__ fstep,
                                                  const int32_t* __restrict__ start, int horizon,
                                                  const int32_t* __restrict__ blkoff,
                                                  int32_t* __restrict__ act, const Ctrl* ctrl) {
  if (ctrl->done) return;
  const int k = blockIdx.x * NT + threadIdx.x;
  const bool a = act_listed(k, n, fstep, start, ctrl->step + horizon);
  const uint64_t m = __ballot(a);
  __shared__ int wc[NT / 64];
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  if (lane == 0) wc[w] = __popcll(m);
  __syncthreads();
  int base = blkoff[blockIdx.x];
  for (int v = 0; v < w; ++v) base += wc[v];
  if (a) act[base + __popcll(m & ((1ull << lane) - 1ull))] = k;
}

// ---- hand-off batch build ---------------------------------------------------------
// Per local slot k of the batch: its volume slot's right neighbour, id and start state;
// gmap takes the local slot of every volume slot in the batch (reset by k_hand_unmap).
__global__ __launch_bounds__(NT) void k_hand_init(int n, const int32_t* __restrict__ gsl,
                                                  const int32_t* __restrict__ start,
                                                  const int32_t* __restrict__ gnext,
                                                  const int64_t* __restrict__ gid,
                                                  int32_t* __restrict__ gnx, int64_t* id,
                                                  int32_t* fstep, int32_t* face, int32_t* lev,
                                                  int32_t* __restrict__ gmap) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n) return;
  const int g = gsl[k];
  gnx[k] = gnext[g];
  id[k] = gid[g];
  fstep[k] = FS_ACTIVE;
  face[k] = -1;
  lev[k] = start[k] - 1;
  gmap[g] = k;
}

// Local links (within one sub-region; others stay -1: their vertices are read from the
// world sheet) and an element-size estimate from each point's first edge.
__global__ __launch_bounds__(NT) void k_hand_links(int n, const int32_t* __restrict__ gsl,
                                                   const int32_t* __restrict__ gnx,
                                                   const int32_t* __restrict__ start,
                                                   const int32_t* __restrict__ gprev,
                                                   const int32_t* __restrict__ gmap,
                                                   const int32_t* __restrict__ rid,
                                                   int32_t* nxt, int32_t* prv, HistCfg hs,
                                                   sp::Period P, Ctrl* ctrl) {
  const int k = blockIdx.x * NT + threadIdx.x;
  uint64_t key = 0;
  if (k < n) {
    const int g = gsl[k];
    int a = gmap[gnx[k]];
    int b = gmap[gprev[g]];
    if (a >= n || b >= n) atomicOr(&ctrl->err, HERR_INPUT);  // (a stale scratch entry)
    if (a >= 0 && (a >= n || rid[a] != rid[k])) a = -1;
    if (b >= 0 && (b >= n || rid[b] != rid[k])) b = -1;
    nxt[k] = a;
    prv[k] = b;
    // element-size estimate (the first grids' cell edge follows it): the spatial box of
    // the point's element of the band below its start slice, when both of that band's
    // slices are built; else twice the distance to its neighbour on the start slice (an
    // element also spans one step of motion: sized by the neighbour distance alone, most
    // first elements would exceed the cells and take the large-element path)
    const int s = start[k];
    if (s - hs.s0 >= 0 && s - hs.s0 < hs.ns) {
      const V4 L = ldh(hs, s, g), R = ldh(hs, s, gnx[k]);
      if (L.t == L.t && R.t == R.t) {
        double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
        auto add = [&](const V4& V) {
          const double d[3] = {V.x - L.x, V.y - L.y, V.z - L.z};
          for (int c = 0; c < 3; ++c) {
            const double w = d[c] - P.box * P.nearest(d[c]);
            lo[c] = fmin(lo[c], w);
            hi[c] = fmax(hi[c], w);
          }
        };
        add(R);
        bool below = false;
        if (s - 1 - hs.s0 >= 0) {
          const V4 B = ldh(hs, s - 1, g), Bj = ldh(hs, s - 1, gnx[k]);
          if (B.t == B.t && Bj.t == Bj.t) {
            add(B);
            add(Bj);
            below = true;
          }
        }
        double e = fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2]));
        if (!below) e *= 2.0;
        key = order_key(e);
      }
    }
  }
  key = wave_max_u64(key);
  if ((threadIdx.x & 63) == 0 && key != 0) atomicMax((unsigned long long*)&ctrl->ext_key, key);
}

__global__ __launch_bounds__(NT) void k_hand_unmap(int n, const int32_t* __restrict__ gsl,
                                                   int32_t* __restrict__ gmap) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k < n) gmap[gsl[k]] = -1;
}

// ---- hand-off run set-up ------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_hist_fill(double4* __restrict__ H, int64_t* __restrict__ home,
                                                  uint64_t m) {
  const uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * NT;
  for (uint64_t q = i; q < m; q += stride) {
    H[q] = make_double4(0.0, 0.0, 0.0, __builtin_nan(""));
    home[q] = HOME_NONE;
  }
}

// The initial surface's two slices into the world sheet; start tokens of the first two
// diamonds each point's left neighbour builds: their bottoms are the point's vertices on
// the two initial slices, so they belong to those vertices' regions.
__global__ __launch_bounds__(NT) void k_hist_ic(const semipar_point_rec* __restrict__ rec, int n,
                                                HistCfg hs, HandTok* __restrict__ tok,
                                                unsigned long long* __restrict__ ntok,
                                                int32_t* __restrict__ err) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  const semipar_point_rec r = rec[j];
  const V4 a{r.x_prev[0], r.x_prev[1], r.x_prev[2], r.x_prev[3]};
  const V4 b{r.x[0], r.x[1], r.x[2], r.x[3]};
  hs.H[j] = make_double4(a.x, a.y, a.z, a.t);
  hs.H[hs.n + j] = make_double4(b.x, b.y, b.z, b.t);
  // the second slice counts as built from the first slice's vertices of j and next j
  const semipar_point_rec rn = rec[hs.gnext[j]];
  const V4 an{rn.x_prev[0], rn.x_prev[1], rn.x_prev[2], rn.x_prev[3]};
  const int64_t na = hist_name(hs, a);
  bool tie = false;
  const int64_t nb = resolve_home(hist_name(hs, b), na, hist_name(hs, an), na, &tie);
  if (tie) atomicOr(err, HERR_TIE);
  hs.home[j] = na;
  hs.home[hs.n + j] = nb;
  const int32_t da = hist_region(hs, na);
  const int32_t db = nb != na ? hist_region(hs, nb) : -1;
  if (da >= 0) {
    const unsigned long long w = atomicAdd(ntok, 1ull);
    tok[w] = HandTok{hs.gprev[j], hs.s0 + 1, da, 0};
  }
  if (db >= 0) {
    const unsigned long long w = atomicAdd(ntok, 1ull);
    tok[w] = HandTok{hs.gprev[j], hs.s0 + 2, db, 0};
  }
}

__global__ __launch_bounds__(NT) void k_emit_count(int n, const int32_t* fstep,
                                                   const semipar_point_rec* frz,
                                                   int32_t* __restrict__ blkcnt) {
  __shared__ int c[4];
  if (threadIdx.x < 4) c[threadIdx.x] = 0;
  __syncthreads();
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k < n) atomicAdd(&c[emit_stream(k, fstep, frz)], 1);
  __syncthreads();
  if (threadIdx.x < 4) blkcnt[4 * blockIdx.x + threadIdx.x] = c[threadIdx.x];
}

// Exclusive scan of the block counts of each stream (one workgroup); tot[f] = totals.
__global__ __launch_bounds__(1024) void k_emit_scan(const int32_t* __restrict__ blkcnt, int nblk,
                                                    int32_t* __restrict__ blkoff,
                                                    int32_t* __restrict__ tot) {
  __shared__ int32_t sh[1024];
  const int t = threadIdx.x;
  const int per = (nblk + 1023) / 1024;
  for (int f = 0; f < 4; ++f) {
    int sum = 0;
    for (int i = 0; i < per; ++i)
      if (t * per + i < nblk) sum += blkcnt[4 * (t * per + i) + f];
    sh[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int add = t >= o ? sh[t - o] : 0;
      __syncthreads();
      sh[t] += add;
      __syncthreads();
    }
    int run = sh[t] - sum;
    for (int i = 0; i < per; ++i)
      if (t * per + i < nblk) {
        blkoff[4 * (t * per + i) + f] = run;
        run += blkcnt[4 * (t * per + i) + f];
      }
    if (t == 1023) tot[f] = sh[1023];
    __syncthreads();
  }
}

// Records in slot order within each stream; stream f starts at base[f] of out.
__global__ __launch_bounds__(NT) void k_emit_write(Slices X, int n, int s, const int32_t* nxt,
                                                   const int32_t* prv, const int64_t* id,
                                                   const int32_t* fstep,
                                                   const semipar_point_rec* frz,
                                                   const int32_t* __restrict__ blkoff,
                                                   const int32_t* __restrict__ tot,
                                                   int32_t act_flags,
                                                   semipar_point_rec* __restrict__ out) {
  __shared__ int32_t sh[4][NT];
  const int t = threadIdx.x;
  const int k = blockIdx.x * NT + t;
  const int f = k < n ? emit_stream(k, fstep, frz) : -1;
  for (int q = 0; q < 4; ++q) sh[q][t] = (f == q) ? 1 : 0;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {
    int add[4];
    for (int q = 0; q < 4; ++q) add[q] = t >= o ? sh[q][t - o] : 0;
    __syncthreads();
    for (int q = 0; q < 4; ++q) sh[q][t] += add[q];
    __syncthreads();
  }
  if (f < 0) return;
  int base = 0;
  for (int q = 0; q < f; ++q) base += tot[q];
  const int pos = base + blkoff[4 * blockIdx.x + f] + sh[f][t] - 1;
  if (fstep && fstep[k] != FS_ACTIVE)
    out[pos] = frz[k];
  else
    out[pos] = current_record(X, k, s, nxt, prv, id, act_flags);
}

// ---- batches of sub-regions: per-sub-region results -------------------------------
// The points of sub-region q occupy the slots sub_off[q] .. sub_off[q+1]-1 (surface
// order), so the records of q on stream f are the slots of q with that stream, in slot
// order. P_f(k) = number of slots before k on stream f (exclusive, over the batch).

// Exclusive in-block counts of the 4 streams before thread t (LDS scan of NT threads).
__device__ __forceinline__ void block_stream_prefix(int f, int32_t (*sh)[NT], int32_t pre[4]) {
  const int t = threadIdx.x;
  for (int q = 0; q < 4; ++q) sh[q][t] = (f == q) ? 1 : 0;
  __syncthreads();
  for (int o = 1; o < NT; o <<= 1) {
    int add[4];
    for (int q = 0; q < 4; ++q) add[q] = t >= o ? sh[q][t - o] : 0;
    __syncthreads();
    for (int q = 0; q < 4; ++q) sh[q][t] += add[q];
    __syncthreads();
  }
  for (int q = 0; q < 4; ++q) pre[q] = sh[q][t] - ((f == q) ? 1 : 0);
}

// P_q at the first slot of every non-empty sub-region: pst[4 * sub + q].
__global__ __launch_bounds__(NT) void k_emit_sub_start(int n, const int32_t* fstep,
                                                       const semipar_point_rec* frz,
                                                       const int32_t* __restrict__ rid,
                                                       const int32_t* __restrict__ blkoff,
                                                       int32_t* __restrict__ pst) {
  __shared__ int32_t sh[4][NT];
  const int k = blockIdx.x * NT + threadIdx.x;
  const int f = k < n ? emit_stream(k, fstep, frz) : -1;
  int32_t pre[4];
  block_stream_prefix(f, sh, pre);
  if (k < n && (k == 0 || rid[k] != rid[k - 1]))
    for (int q = 0; q < 4; ++q) pst[4 * rid[k] + q] = blkoff[4 * blockIdx.x + q] + pre[q];
}

// Record of slot k to tmp[dst[4 * sub + f] + P_f(k) - pst[4 * sub + f]].
__global__ __launch_bounds__(NT) void k_emit_sub_write(Slices X, int n, int s, const int32_t* nxt,
                                                       const int32_t* prv, const int64_t* id,
                                                       const int32_t* fstep,
                                                       const semipar_point_rec* frz,
                                                       const int32_t* __restrict__ rid,
                                                       const int32_t* __restrict__ blkoff,
                                                       const int32_t* __restrict__ pst,
                                                       const int64_t* __restrict__ dst,
                                                       semipar_point_rec* __restrict__ out) {
  __shared__ int32_t sh[4][NT];
  const int k = blockIdx.x * NT + threadIdx.x;
  const int f = k < n ? emit_stream(k, fstep, frz) : -1;
  int32_t pre[4];
  block_stream_prefix(f, sh, pre);
  if (f < 0) return;
  const int q = rid[k];
  const int64_t pos = dst[4 * q + f] + (blkoff[4 * blockIdx.x + f] + pre[f] - pst[4 * q + f]);
  if (fstep[k] != FS_ACTIVE)
    out[pos] = frz[k];
  else
    out[pos] = current_record(X, k, s, nxt, prv, id, SEMIPAR_FLAG_ACTIVE);
}

// Per sub-region: point-steps (sum over its points of the slices advanced) and the
// largest number of slices any of its points advanced.
__global__ __launch_bounds__(NT) void k_sub_stats(int n, const int32_t* __restrict__ fstep,
                                                  int32_t cur, int32_t step0,
                                                  const int32_t* __restrict__ rid,
                                                  unsigned long long* __restrict__ psteps,
                                                  int32_t* __restrict__ smax,
                                                  const int32_t* __restrict__ start) {
  const int k = blockIdx.x * NT + threadIdx.x;
  const bool live = k < n;
  const int q = live ? (rid ? rid[k] : 0) : -1;
  int adv = 0;
  if (live) {
    // a hand-off batch's points start at their own steps
    adv = (fstep[k] == FS_ACTIVE ? cur : fstep[k]) - (start ? start[k] : step0);
    adv = adv < 0 ? 0 : adv;
  }
  if (wave_uniform(q, live)) {
    unsigned long long sum = (unsigned long long)adv;
    int mx = adv;
    for (int o = 32; o > 0; o >>= 1) {
      sum += __shfl_xor(sum, o, 64);
      const int w = __shfl_xor(mx, o, 64);
      mx = w > mx ? w : mx;
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&psteps[q], sum);
      atomicMax(&smax[q], mx);
    }
  } else if (live) {
    atomicAdd(&psteps[q], (unsigned long long)adv);
    atomicMax(&smax[q], adv);
  }
}

// ---- cost-model features of the initial surface of each sub-region ----------------
constexpr int FEAT_GRID = 16;  // cells per side of the occupancy grid of a region
constexpr int FEAT_CELLS = FEAT_GRID * FEAT_GRID * FEAT_GRID;
constexpr int FEAT_ACC = 5;  // sum v^2, count, sum edge, count, open pieces
constexpr int FEAT_STRIDE = 16;  // one cache line per region's sums (their atomics do not share)
static_assert(FEAT_ACC <= FEAT_STRIDE, "feature sums fit one line");

// Per point of the current surface (before any step): transverse speed of the diamond
// at k (spatial (L-B)+(R-B) over its time extent), length of the edge to next[k] on
// the current slice, open-piece starts (no prev), and the occupancy of a 16^3 grid
// over the spatial cube of side 2g around the region's centre.
// One point's share of its sub-region's feature sums (every lane of the wave calls it):
// L its vertex on the current slice; with a right neighbour (has_j), R and B that
// neighbour's vertices on the current and previous slices; open: no left neighbour.
__device__ __forceinline__ void feat_accumulate(bool live, int q, const V4& L, bool has_j,
                                                const V4& R, const V4& B, bool open_,
                                                const RegionGeom* __restrict__ geoms,
                                                const sp::Period& P, double* __restrict__ acc,
                                                int32_t* __restrict__ grid) {
  double v2 = 0.0, nv = 0.0, e = 0.0, ne = 0.0, open = 0.0;
  if (live) {
    if (has_j) {
      const double ax = sp::min_image(L.x - B.x, P), ay = sp::min_image(L.y - B.y, P),
                   az = sp::min_image(L.z - B.z, P);
      const double vx = ax + (R.x - B.x), vy = ay + (R.y - B.y), vz = az + (R.z - B.z);
      const double dt = (L.t - B.t) + (R.t - B.t);
      if (dt > 0.0) {
        v2 = (vx * vx + vy * vy + vz * vz) / (dt * dt);
        nv = 1.0;
      }
      const double ex = sp::min_image(R.x - L.x, P), ey = sp::min_image(R.y - L.y, P),
                   ez = sp::min_image(R.z - L.z, P);
      e = sqrt(ex * ex + ey * ey + ez * ez);
      ne = 1.0;
    }
    if (open_) open = 1.0;
    const RegionGeom& G = geoms[q];
    const double g = 0.5 / G.inv2g;
    double ctr[3];
    region_centre(G, ctr);
    const double c[3] = {sp::min_image(L.x - ctr[0], P), sp::min_image(L.y - ctr[1], P),
                         sp::min_image(L.z - ctr[2], P)};
    int ci[3];
    for (int a = 0; a < 3; ++a) {
      const int v = (int)floor((c[a] + g) * (FEAT_GRID / (2.0 * g)));
      ci[a] = v < 0 ? 0 : (v >= FEAT_GRID ? FEAT_GRID - 1 : v);
    }
    atomicAdd(&grid[(int64_t)q * FEAT_CELLS + (ci[0] * FEAT_GRID + ci[1]) * FEAT_GRID + ci[2]], 1);
  }
  double* a = acc + (int64_t)FEAT_STRIDE * (q < 0 ? 0 : q);
  if (wave_uniform(q, live)) {
    for (int o = 32; o > 0; o >>= 1) {
      v2 += __shfl_xor(v2, o, 64);
      nv += __shfl_xor(nv, o, 64);
      e += __shfl_xor(e, o, 64);
      ne += __shfl_xor(ne, o, 64);
      open += __shfl_xor(open, o, 64);
    }
    if ((threadIdx.x & 63) != 0) return;
  } else if (!live) {
    return;
  }
  atomicAdd(&a[0], v2);
  atomicAdd(&a[1], nv);
  atomicAdd(&a[2], e);
  atomicAdd(&a[3], ne);
  atomicAdd(&a[4], open);
}

__global__ __launch_bounds__(NT) void k_feat_points(Slices X, int n, int s,
                                                    const int32_t* __restrict__ nxt,
                                                    const int32_t* __restrict__ prv,
                                                    const int32_t* __restrict__ rid,
                                                    const RegionGeom* __restrict__ geoms,
                                                    sp::Period P, double* __restrict__ acc,
                                                    int32_t* __restrict__ grid) {
  const int k = blockIdx.x * NT + threadIdx.x;
  const bool live = k < n;
  const int q = live ? rid[k] : -1;
  V4 L{}, R{}, B{};
  bool has_j = false, open_ = false;
  if (live) {
    const int ic = s % 3, ip = (s + 2) % 3;
    L = ld(X, ic, k);
    const int j = nxt[k];
    if (j >= 0) {
      R = ld(X, ic, j);
      B = ld(X, ip, j);
      has_j = true;
    }
    open_ = prv[k] < 0;
  }
  feat_accumulate(live, q, L, has_j, R, B, open_, geoms, P, acc, grid);
}

// The same sums straight from the surfaces of a tiling (device memory, read in place):
// point k of the concatenation lies in region q = region_of(k) at k - off[q].
__device__ __forceinline__ int region_of(const int64_t* __restrict__ off, int nr, int64_t k) {
  int lo = 0, hi = nr - 1;  // off[lo] <= k < off[hi + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(NT) void k_featsurf_insert(
    const semipar_point_rec* const* __restrict__ srf, const int64_t* __restrict__ off, int nr,
    int n, int64_t* __restrict__ hkey, int32_t* __restrict__ hval, uint32_t hmask,
    int32_t* __restrict__ err) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k >= n) return;
  const int q = region_of(off, nr, k);
  const int64_t id = srf[q][k - off[q]].id;
  if (id == ID_EMPTY) {
    atomicOr(err, 1);
    return;
  }
  uint32_t h = id_hash(id, hmask);
  for (uint32_t probe = 0; probe <= hmask; ++probe) {
    const unsigned long long prev = atomicCAS((unsigned long long*)&hkey[h],
                                              (unsigned long long)ID_EMPTY, (unsigned long long)id);
    if ((int64_t)prev == ID_EMPTY) {
      hval[h] = k;
      return;
    }
    if ((int64_t)prev == id) {
      atomicOr(err, 2);  // duplicate id
      return;
    }
    h = (h + 1) & hmask;
  }
  atomicOr(err, 4);
}

__global__ __launch_bounds__(NT) void k_featsurf_points(
    const semipar_point_rec* const* __restrict__ srf, const int64_t* __restrict__ off, int nr,
    int n, const int64_t* __restrict__ hkey, const int32_t* __restrict__ hval, uint32_t hmask,
    const RegionGeom* __restrict__ geoms, sp::Period P, double* __restrict__ acc,
    int32_t* __restrict__ grid) {
  const int k = blockIdx.x * NT + threadIdx.x;
  const bool live = k < n;
  int q = -1;
  V4 L{}, R{}, B{};
  bool has_j = false, open_ = false;
  if (live) {
    q = region_of(off, nr, k);
    const semipar_point_rec& r = srf[q][k - off[q]];
    L = V4{r.x[0], r.x[1], r.x[2], r.x[3]};
    // a neighbour in another region's surface is absent, as in that region alone
    const int j = id_lookup(hkey, hval, hmask, r.next_id);
    const int qj = j >= 0 ? region_of(off, nr, j) : -1;
    if (qj == q) {
      const semipar_point_rec& rj = srf[qj][j - off[qj]];
      R = V4{rj.x[0], rj.x[1], rj.x[2], rj.x[3]};
      B = V4{rj.x_prev[0], rj.x_prev[1], rj.x_prev[2], rj.x_prev[3]};
      has_j = true;
    }
    const int pk = id_lookup(hkey, hval, hmask, r.prev_id);
    open_ = pk < 0 || region_of(off, nr, pk) != q;
  }
  feat_accumulate(live, q, L, has_j, R, B, open_, geoms, P, acc, grid);
}

// One workgroup per sub-region: the 12 features (FP32).
//   0 log1p(points)   1 log1p(open pieces)   2 RMS transverse speed
//   3..10 fraction of the points in cells whose occupancy, relative to the mean over
//         the 16^3 grid, falls in log2 bin b (b = floor(log2(rel)) + 4, clamped to 0..7)
//   11 log1p(mean edge length / region size)
__global__ __launch_bounds__(256) void k_feat_final(const int32_t* __restrict__ grid,
                                                    const double* __restrict__ acc,
                                                    const int64_t* __restrict__ npts,
                                                    const RegionGeom* __restrict__ geoms,
                                                    float* __restrict__ feat) {
  __shared__ unsigned long long hist[8];
  const int q = blockIdx.x;
  const int t = threadIdx.x;
  if (t < 8) hist[t] = 0;
  __syncthreads();
  const int64_t nq = npts[q];
  if (nq > 0)
    for (int c = t; c < FEAT_CELLS; c += 256) {
      const int occ = grid[(int64_t)q * FEAT_CELLS + c];
      if (occ == 0) continue;
      const double rel = (double)occ * FEAT_CELLS / (double)nq;
      int b = (int)floor(log2(rel)) + 4;
      b = b < 0 ? 0 : (b > 7 ? 7 : b);
      atomicAdd(&hist[b], (unsigned long long)occ);
    }
  __syncthreads();
  if (t == 0) {
    float* f = feat + 12 * (int64_t)q;
    const double* a = acc + (int64_t)FEAT_STRIDE * q;
    const double size = 1.4142135623730951 * 0.5 / geoms[q].inv2g;
    f[0] = (float)log1p((double)nq);
    f[1] = (float)log1p(a[4]);
    f[2] = (float)(a[1] > 0.0 ? sqrt(a[0] / a[1]) : 0.0);
    for (int b = 0; b < 8; ++b) f[3 + b] = nq > 0 ? (float)((double)hist[b] / (double)nq) : 0.f;
    f[11] = (float)(a[3] > 0.0 ? log1p(a[2] / a[3] / size) : 0.0);
  }
}

// ---- event log of a batch: order (sub-region, step, t*, id_a, id_b) ---------------
// Candidate slot pairs -> (smaller id, larger id).
__global__ __launch_bounds__(NT) void k_cand_ids(const int2* __restrict__ cand, int64_t n,
                                                 const int64_t* __restrict__ id,
                                                 int64_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= n) return;
  const int64_t a = id[cand[i].x], b = id[cand[i].y];
  out[2 * i] = a < b ? a : b;
  out[2 * i + 1] = a < b ? b : a;
}


// Sort of a batch's event log into listing order per sub-region: (sub-region, step,
// t*, id_a, id_b), a total order (a pair of elements meets at most once per step). A
// bitonic sort over a power-of-two array of 24-byte keys: hi = (sub-region << 32 | step),
// mid = order key of t*, and the event's index, whose ids decide equal (hi, mid).
struct EvKey {
  uint64_t hi, mid;
  int32_t idx;
  int32_t pad;
};
constexpr int EVS_LDS = 1024;  // keys sorted in LDS per workgroup (strides below this)

__device__ __forceinline__ bool evkey_less(const EvKey& x, const EvKey& y,
                                           const semipar_event* __restrict__ log) {
  if (x.hi != y.hi) return x.hi < y.hi;
  if (x.mid != y.mid) return x.mid < y.mid;
  if (x.idx < 0 || y.idx < 0) return x.idx > y.idx;  // padding (idx -1) sorts last
  const semipar_event& a = log[x.idx];
  const semipar_event& b = log[y.idx];
  if (a.id_a != b.id_a) return a.id_a < b.id_a;
  return a.id_b < b.id_b;
}

__global__ __launch_bounds__(NT) void k_ev_keys(const semipar_event* __restrict__ log,
                                                const int32_t* __restrict__ lrid, int64_t n,
                                                int64_t npow, EvKey* __restrict__ keys) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= npow) return;
  EvKey k;
  if (i < n) {
    k.hi = ((uint64_t)(uint32_t)lrid[i] << 32) | (uint32_t)log[i].step;
    k.mid = order_key(log[i].t_star);
    k.idx = (int32_t)i;
  } else {
    k.hi = KEY_MAX;
    k.mid = KEY_MAX;
    k.idx = -1;
  }
  k.pad = 0;
  keys[i] = k;
}

// Compare-exchange of element i with i ^ j in the bitonic merge of size kk (ascending
// where i & kk == 0).
__device__ __forceinline__ void evkey_cx(EvKey* v, int64_t i, int64_t j, int64_t kk,
                                         const semipar_event* __restrict__ log) {
  const int64_t l = i ^ j;
  if (l <= i) return;
  const bool up = (i & kk) == 0;
  const EvKey a = v[i], b = v[l];
  const bool sw = up ? evkey_less(b, a, log) : evkey_less(a, b, log);
  if (sw) {
    v[i] = b;
    v[l] = a;
  }
}

// One global stage (stride j >= EVS_LDS) of the merge of size kk.
__global__ __launch_bounds__(NT) void k_ev_bitonic(EvKey* __restrict__ keys, int64_t npow,
                                                   int64_t kk, int64_t j,
                                                   const semipar_event* __restrict__ log) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i < npow) evkey_cx(keys, i, j, kk, log);
}

// Every stage with stride below EVS_LDS, in LDS, for merges of size kk0 .. kk1 (kk1 <=
// EVS_LDS: the whole sort of each block; kk0 = kk1 > EVS_LDS: the tail of one merge).
__global__ __launch_bounds__(NT) void k_ev_bitonic_lds(EvKey* __restrict__ keys, int64_t kk0,
                                                       int64_t kk1,
                                                       const semipar_event* __restrict__ log) {
  __shared__ EvKey v[EVS_LDS];
  const int64_t base = (int64_t)blockIdx.x * EVS_LDS;
  for (int i = threadIdx.x; i < EVS_LDS; i += NT) v[i] = keys[base + i];
  __syncthreads();
  for (int64_t kk = kk0; kk <= kk1; kk <<= 1) {
    for (int64_t j = (kk > EVS_LDS ? EVS_LDS : kk) >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < EVS_LDS; i += NT) {
        const int l = i ^ (int)j;
        if (l > i) {
          const bool up = ((base + i) & kk) == 0;
          const EvKey a = v[i], b = v[l];
          const bool sw = up ? evkey_less(b, a, log) : evkey_less(a, b, log);
          if (sw) {
            v[i] = b;
            v[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < EVS_LDS; i += NT) keys[base + i] = v[i];
}

__global__ __launch_bounds__(NT) void k_ev_gather(const semipar_event* __restrict__ log,
                                                  const int32_t* __restrict__ lrid,
                                                  const EvKey* __restrict__ keys, int64_t n,
                                                  semipar_event* __restrict__ out,
                                                  int32_t* __restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  const bool live = i < n;
  int32_t q = -1;
  if (live) {
    const int32_t e = keys[i].idx;
    out[i] = log[e];
    q = lrid[e];
  }
  // The events are in sub-region order, so a wave holds a few runs of equal sub-region:
  // one counter update per run (per-event atomics on a few cache lines serialise).
  const int lane = (int)(threadIdx.x & 63);
  const int32_t qp = __shfl_up(q, 1, 64);
  const bool head = live && (lane == 0 || qp != q);
  const uint64_t heads = __ballot(head);
  const int n_live = __popcll(__ballot(live));
  if (head) {
    const uint64_t above = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
    const int end = above ? __ffsll((unsigned long long)above) - 1 : n_live;
    atomicAdd(&cnt[q], end - lane);
  }
}

// ---------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------
thread_local char g_last_error[256] = "";

inline int hip_fail(hipError_t e, const char* what, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s failed at semipar.hip:%d: %s", what, line,
           hipGetErrorString(e));
  return SEMIPAR_E_HIP;
}

// A failed device allocation: the place and the device's free memory, for
// semipar_last_error, and SEMIPAR_E_OOM.
inline int oom(int line) {
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  (void)hipGetLastError();
  snprintf(g_last_error, sizeof(g_last_error),
           "device allocation failed at semipar.hip:%d (%.1f of %.1f GiB free)", line,
           fr / 1073741824.0, tot / 1073741824.0);
  return oom(__LINE__);
}

#define RCCHK(x)              \
  do {                        \
    int rc_ = (x);            \
    if (rc_ != 0) return rc_; \
  } while (0)

#define HIPCHK(x)                                          \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__); \
  } while (0)

inline void dfree(void* p) {
  if (p) (void)hipFree(p);
}

template <class T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, sizeof(T) * count);
}

inline int blocks(int64_t n, int nt = NT) { return (int)((n + nt - 1) / nt); }

// Stream-ordered temporaries: allocated and released in order on one stream, so that
// building a region never waits for other streams' work (hipFree would wait for the
// whole device).
template <class T>
hipError_t salloc(T** p, size_t count, hipStream_t s) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMallocAsync((void**)p, sizeof(T) * count, s);
}
inline void sfree(void* p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

}  // namespace

struct semipar_region {
  int64_t n = 0, cap = 0;
  bool bounded = false;
  // buffers replaced by larger ones while the region is in use: released with it, since
  // hipFree waits for the whole device (other lanes' batches included)
  std::vector<void*> retired;
  RegionGeom geom{};
  int32_t n_sub = 0;
  RegionGeom* geoms = nullptr;  // batch: geometry of each sub-region
  int32_t* rid = nullptr;       // batch: sub-region of each point
  std::vector<int64_t> sub_off;  // batch: first slot of each sub-region (n_sub + 1 entries)
  int32_t* log_rid = nullptr;    // batch: sub-region of each logged event
  RCell* rcell = nullptr;        // batch: local grid of each sub-region
  uint64_t* rext = nullptr;      // batch: largest element extent per sub-region (key), one
                                 // entry per REXT_STRIDE words
  double rc_fixed_h = 0.0;       // batch: fixed cell edge (0 = adaptive)
  double p_ic = 1.0;             // intercommutation probability (the resolve launch carries it)
  uint64_t seed = 0;             // key of the crossings' draws
  int32_t step0 = 1;             // slice index of the initial surfaces
  int32_t *fstep = nullptr, *face = nullptr;  // bounded: stop step and exit face per point
  uint8_t* wlive = nullptr;  // per 64 slots: 1 while one of them may still advance
  semipar_point_rec* frz = nullptr;           // bounded: record of each stopped point
  int cosmology = 0;
  double hcoef = 0.0, box = 1.0;
  hipStream_t stream = nullptr;
  sp::Period P{};
  uint64_t* blkred = nullptr;  // per block: min t of the slice being written, max extent
  Slices X{};
  int32_t *nxt = nullptr, *prv = nullptr;
  int64_t* id = nullptr;
  Ctrl* ctrl = nullptr;
  Ctrl* ctrl_h = nullptr;  // pinned mirror
  double ext0 = 0.0;       // initial element-size estimate
  // step buffers (configured per evolve parameters)
  int screen = -1;
  void* ebox = nullptr;
  int32_t* ecell = nullptr;
  LargeBox* large = nullptr;
  HashCfg hc{};
  int32_t *cnt = nullptr, *loc = nullptr, *tile_tot = nullptr, *toff = nullptr;
  int2* sent = nullptr;                      // cell-sorted (cell, slot) of each element
  void* sbox = nullptr;                      // cell-sorted screen boxes
  int ntiles = 0;
  int2* cand = nullptr;
  int64_t cap_cand = 0;
  EvCand* ev = nullptr;
  int64_t cap_evt = 0;
  uint64_t* best = nullptr;
  int32_t* used = nullptr;
  int8_t* evs = nullptr;
  semipar_event* log = nullptr;
  int64_t log_cap = 0;
  bool broken = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool own_stream = false;
  hipGraphExec_t gexec = nullptr;
  int g_steps = 0;
  int g_timed = -1;
  bool cells_set = false;  // the device grid has been chosen (adaptive runs keep it)
  int split = N_PENCIL;    // screen variant: threads per element (1 or 5), or SPLIT_PRE
  PencilAux* saux = nullptr;  // SPLIT_PRE: neighbour pencils of each sorted element
  int64_t* dsub_off = nullptr;  // persistent launches: first slot of each sub-region
  int32_t* pb_head = nullptr;   // persistent launches: the next sub-region to take
  bool cells_fixed = false;
  // measurement: HIP events around every launch of one kernel (timed_kernel)
  int timed = -1;
  std::vector<hipEvent_t> tev;
  // loop record and removal
  int32_t* lev = nullptr;  // step of the last accepted event touching each point's element
  bool removed = false;    // a loop was removed: whole-volume kernels then read fstep
  int32_t *lab[2] = {nullptr, nullptr}, *lptr[2] = {nullptr, nullptr};  // list ranking
  int32_t *lcnt = nullptr, *levm = nullptr, *lbad = nullptr;  // per chain (lowest slot)
  int32_t *lidx = nullptr, *lrep = nullptr;  // chain -> loop index, loop index -> chain
  int32_t* lctr = nullptr;                   // loops and points of one check
  int32_t* lctr_h = nullptr;                 // pinned mirror
  double* lacc = nullptr;                    // per loop of one check: energy, centre sums
  int64_t lacc_cap = 0;
  semipar_loop* llog = nullptr;  // loop log (completion order within a check)
  int32_t* llog_rid = nullptr;   // sub-region of each logged loop (batches; else 0)
  int64_t llog_n = 0, llog_cap = 0;
  // hand-off batch of a tiling run: the world sheet and the tiling's names are the
  // caller's; the per-point tables and the token buffer are the region's
  bool hist = false;
  HistCfg hcfg{};
  // bounded region: the points still advancing at the start of each block of steps, in
  // ascending slot order (the per-point kernels walk it), and its per-block counts
  int32_t *act = nullptr, *actblk = nullptr;
  int32_t act_last = INT32_MIN;  // eager blocks: the last step the current list covers
  int32_t *hgsl = nullptr, *hgnx = nullptr, *hstart = nullptr;
  int64_t* hsname = nullptr;
  HandTok* htok = nullptr;
};

namespace {

void free_step_buffers(semipar_region* r) {
  dfree(r->ebox);
  dfree(r->ecell);
  dfree(r->large);
  dfree(r->cnt);
  dfree(r->loc);
  dfree(r->tile_tot);
  dfree(r->toff);
  dfree(r->sent);
  dfree(r->sbox);
  dfree(r->cand);
  dfree(r->ev);
  dfree(r->best);
  dfree(r->used);
  dfree(r->evs);
  dfree(r->saux);
  r->saux = nullptr;
  r->ebox = nullptr;
  r->ecell = r->cnt = r->loc = r->tile_tot = r->toff = r->used = nullptr;
  r->sent = nullptr;
  r->sbox = nullptr;
  r->large = nullptr;
  r->cand = nullptr;
  r->ev = nullptr;
  r->best = nullptr;
  r->evs = nullptr;
  r->screen = -1;
  r->cap_cand = r->cap_evt = 0;
}

void drop_graph(semipar_region* r) {
  if (r->gexec) (void)hipGraphExecDestroy(r->gexec);
  r->gexec = nullptr;
  r->g_steps = 0;
  r->g_timed = -1;
}

int ensure_timing_events(semipar_region* r, int K) {
  while ((int)r->tev.size() < 2 * K) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    r->tev.push_back(e);
  }
  return SEMIPAR_OK;
}

inline void mark(semipar_region* r, int kid, int slot) {
  if (r->timed == kid) (void)hipEventRecord(r->tev[slot], r->stream);
}

uint64_t next_pow2(uint64_t v) {
  uint64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

HashCfg make_hash(const semipar_region* r) {
  HashCfg hc{};
  const double box = r->box;
  uint64_t B = next_pow2(std::max<uint64_t>(2 * (uint64_t)std::max<int64_t>(r->cap, 1), TS));
  if (B > (uint64_t)TS * MAX_TILES) B = (uint64_t)TS * MAX_TILES;
  hc.B = (int32_t)B;
  hc.bmask = (uint32_t)(B - 1);
  hc.tol = box * std::ldexp(1.0, -30);
  hc.tolL = box * std::ldexp(1.0, -24);
  hc.tref = 0.0;
  hc.tol_t = std::ldexp(1.0, -30) * 64.0;
  return hc;
}

int configure(semipar_region* r, const semipar_evolve_params* p) {
  const int screen = p->screen == SEMIPAR_SCREEN_F32 ? 2 : 1;
  const double capd = (double)std::max<int64_t>(r->cap, 1);
  const int64_t want_cand = p->cand_per_point > 0
                                ? (int64_t)std::ceil(p->cand_per_point * capd) + 64
                                : (int64_t)(4.0 * capd) + 65536;
  const int64_t want_evt = p->events_per_point > 0
                               ? (int64_t)std::ceil(p->events_per_point * capd) + 64
                               : (int64_t)(0.5 * capd) + 65536;
  if (r->screen == screen && r->cap_cand >= want_cand && r->cap_evt >= want_evt)
    return SEMIPAR_OK;
  const int64_t old_cand = r->cap_cand, old_evt = r->cap_evt;
  drop_graph(r);
  free_step_buffers(r);
  const int64_t cap = std::max<int64_t>(r->cap, 1);
  r->hc = make_hash(r);
  r->ntiles = r->hc.B / TS;
  HIPCHK(hipMalloc(&r->ebox, (size_t)cap * 8 * (screen == 1 ? sizeof(double) : sizeof(float))));
  HIPCHK(dalloc(&r->ecell, cap));
  // points that have stopped are never visited again: their cell must read NO_ELEM
  k_fill_i32<<<blocks(cap), NT, 0, r->stream>>>(r->ecell, (uint64_t)cap, NO_ELEM);
  HIPCHK(hipGetLastError());
  HIPCHK(dalloc(&r->large, cap));
  HIPCHK(dalloc(&r->cnt, r->hc.B));
  HIPCHK(dalloc(&r->loc, (size_t)r->hc.B + 1));
  HIPCHK(dalloc(&r->tile_tot, r->ntiles));
  HIPCHK(dalloc(&r->toff, (size_t)r->ntiles + 1));
  HIPCHK(dalloc(&r->sent, cap));
  HIPCHK(hipMalloc(&r->sbox, (size_t)cap * 8 * (screen == 1 ? sizeof(double) : sizeof(float))));
  HIPCHK(hipMemsetAsync(r->cnt, 0, sizeof(int32_t) * r->hc.B, r->stream));
  HIPCHK(hipMemsetAsync(r->loc, 0, sizeof(int32_t) * ((size_t)r->hc.B + 1), r->stream));
  r->cap_cand = std::max(want_cand, old_cand);
  r->cap_evt = std::max(want_evt, old_evt);
  if (r->cap_cand > INT32_MAX / 2) r->cap_cand = INT32_MAX / 2;
  if (r->cap_evt > INT32_MAX / 2) r->cap_evt = INT32_MAX / 2;
  HIPCHK(dalloc(&r->cand, r->cap_cand));
  HIPCHK(dalloc(&r->ev, r->cap_evt));
  HIPCHK(dalloc(&r->evs, r->cap_evt));
  HIPCHK(dalloc(&r->best, cap));
  HIPCHK(dalloc(&r->used, cap));
  HIPCHK(hipMemsetAsync(r->best, 0, sizeof(uint64_t) * cap, r->stream));
  HIPCHK(hipMemsetAsync(r->used, 0, sizeof(int32_t) * cap, r->stream));
  r->screen = screen;
  // the region's own stream only: other regions' work on other streams goes on
  HIPCHK(hipStreamSynchronize(r->stream));
  return SEMIPAR_OK;
}

int ensure_log(semipar_region* r, int64_t need) {
  if (r->log_cap >= need) return SEMIPAR_OK;
  int64_t nc = std::max<int64_t>(need, std::max<int64_t>(2 * r->log_cap, 1 << 16));
  semipar_event* nl = nullptr;
  HIPCHK(hipMalloc(&nl, sizeof(semipar_event) * nc));
  if (r->log && r->ctrl_h->log_n > 0)
    HIPCHK(hipMemcpyAsync(nl, r->log, sizeof(semipar_event) * r->ctrl_h->log_n,
                          hipMemcpyDeviceToDevice, r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  if (r->rid) {
    int32_t* nr = nullptr;
    HIPCHK(hipMalloc(&nr, sizeof(int32_t) * nc));
    if (r->log_rid && r->ctrl_h->log_n > 0)
      HIPCHK(hipMemcpyAsync(nr, r->log_rid, sizeof(int32_t) * r->ctrl_h->log_n,
                            hipMemcpyDeviceToDevice, r->stream));
    HIPCHK(hipStreamSynchronize(r->stream));
    if (r->log_rid) r->retired.push_back(r->log_rid);
    r->log_rid = nr;
  }
  if (r->log) r->retired.push_back(r->log);
  r->log = nl;
  r->log_cap = nc;
  drop_graph(r);
  return SEMIPAR_OK;
}

// Hand-off batch: room for `need` start tokens (the written ones are kept).
int ensure_tokens(semipar_region* r, int64_t need) {
  if (r->hcfg.tok_cap >= need && r->htok) return SEMIPAR_OK;
  const int64_t nc = std::max<int64_t>(need, std::max<int64_t>(2 * r->hcfg.tok_cap, 1 << 16));
  HandTok* nt = nullptr;
  HIPCHK(dalloc(&nt, (size_t)nc));
  const int64_t have = std::min<int64_t>(r->ctrl_h->tok_n, r->hcfg.tok_cap);
  if (r->htok && have > 0)
    HIPCHK(hipMemcpyAsync(nt, r->htok, sizeof(HandTok) * have, hipMemcpyDeviceToDevice,
                          r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  if (r->htok) r->retired.push_back(r->htok);
  r->htok = nt;
  r->hcfg.tok = nt;
  r->hcfg.tok_cap = nc;
  drop_graph(r);  // the step launches carry the buffer
  return SEMIPAR_OK;
}

// A deferred step reported that the candidate (bit 1) or event (bit 2) buffer was too
// small: double it. The step is then taken again from the same state.
int grow_step_caps(semipar_region* r, int defer) {
  drop_graph(r);
  HIPCHK(hipStreamSynchronize(r->stream));
  if (defer & 1) {
    if (r->cap_cand >= INT32_MAX / 4) return SEMIPAR_E_OVERFLOW;
    r->retired.push_back(r->cand);
    r->cand = nullptr;
    r->cap_cand *= 2;
    HIPCHK(dalloc(&r->cand, r->cap_cand));
  }
  if (defer & 2) {
    if (r->cap_evt >= INT32_MAX / 4) return SEMIPAR_E_OVERFLOW;
    r->retired.push_back(r->ev);
    r->retired.push_back(r->evs);
    r->ev = nullptr;
    r->evs = nullptr;
    r->cap_evt *= 2;
    HIPCHK(dalloc(&r->ev, r->cap_evt));
    HIPCHK(dalloc(&r->evs, r->cap_evt));
  }
  return SEMIPAR_OK;
}

template <bool FRW, int SCR, bool BND, bool HIST>
void launch_evolve_t(semipar_region* r, int n, int nb) {
  k_evolve<FRW, SCR, BND, HIST><<<nb, NT, 0, r->stream>>>(
      r->X, r->nxt, r->prv, r->id, n, r->P, r->hcoef, r->ctrl, r->hc, r->ebox, r->ecell,
      r->cnt, r->large, r->blkred, (BND || r->removed) ? r->fstep : nullptr, r->face, r->frz,
      r->geom, r->geoms, r->rid, r->rcell, r->rext, r->wlive, r->hcfg, r->act);
}

template <bool FRW, bool BND, bool HIST>
void launch_evolve_s(semipar_region* r, int scr, int n, int nb) {
  if (scr == 0) launch_evolve_t<FRW, 0, BND, HIST>(r, n, nb);
  else if (scr == 1) launch_evolve_t<FRW, 1, BND, HIST>(r, n, nb);
  else launch_evolve_t<FRW, 2, BND, HIST>(r, n, nb);
}

// Diamond tops (+ element data when scr != 0) of one step.
void launch_evolve(semipar_region* r, bool frw, int scr, bool bnd, int n, int nb) {
  if (r->hist) {
    if (frw) launch_evolve_s<true, true, true>(r, scr, n, nb);
    else launch_evolve_s<false, true, true>(r, scr, n, nb);
  } else if (frw) {
    if (bnd) launch_evolve_s<true, true, false>(r, scr, n, nb);
    else launch_evolve_s<true, false, false>(r, scr, n, nb);
  } else {
    if (bnd) launch_evolve_s<false, true, false>(r, scr, n, nb);
    else launch_evolve_s<false, false, false>(r, scr, n, nb);
  }
}

template <int SCR, int G>
void launch_screen_t(semipar_region* r, int n, int nb) {
  // chunks covering n elements at most (hashed + large <= n), at most SCREEN_GRID
  // workgroups walking them
  const int nl = G == 1 ? nb : (int)((n + (NT / 64) * SCREEN_EPW - 1) / ((NT / 64) * SCREEN_EPW));
  k_screen<SCR, G><<<xcd_grid(std::min(nl, SCREEN_GRID)), NT, 0, r->stream>>>(
      n, r->sent, r->sbox, r->ebox, r->nxt, r->prv, r->loc, r->toff, r->ntiles, r->large, r->hc,
      r->P, r->cand, (int)r->cap_cand, r->ctrl, r->rid, r->rcell);
}

template <int SCR>
void launch_screen_flat_t(semipar_region* r, int n, int nb) {
  k_screen_flat<SCR><<<xcd_grid(std::min(nb, SCREEN_GRID)), NT, 0, r->stream>>>(
      n, r->sent, r->sbox, r->ebox, r->nxt, r->prv, r->loc, r->toff, r->ntiles, r->large, r->hc,
      r->P, r->cand, (int)r->cap_cand, r->ctrl, r->rid, r->rcell);
  k_screen_large<SCR><<<LARGE_GRID, NT, 0, r->stream>>>(
      r->sent, r->sbox, r->nxt, r->prv, r->loc, r->toff, r->ntiles, r->large, r->hc, r->P,
      r->cand, (int)r->cap_cand, r->ctrl, r->rid, r->rcell);
}

template <int SCR>
void launch_screen_pre_t(semipar_region* r, int n, int nb) {
  k_screen_pre<SCR><<<xcd_grid(std::min(nb, SCREEN_GRID)), NT, 0, r->stream>>>(
      n, r->sent, r->sbox, r->ebox, r->saux, r->loc, r->toff, r->ntiles, r->large, r->hc, r->P,
      r->cand, (int)r->cap_cand, r->ctrl, r->rid, r->rcell, r->nxt, r->prv);
}

// Screen launch: precision (FP64 / FP32 boxes) and variant (one or five threads per
// element, or pencils precomputed by k_scatter).
void launch_screen(semipar_region* r, int n, int nb) {
  if (r->split == SPLIT_PRE) {
    if (r->screen == 1) launch_screen_pre_t<1>(r, n, nb);
    else launch_screen_pre_t<2>(r, n, nb);
    return;
  }
  const bool one = r->split == 1;
  if (r->screen == 1) {
    if (one) launch_screen_flat_t<1>(r, n, nb);
    else launch_screen_t<1, N_PENCIL>(r, n, nb);
  } else {
    if (one) launch_screen_flat_t<2>(r, n, nb);
    else launch_screen_t<2, N_PENCIL>(r, n, nb);
  }
}

// Issue one lattice step (all kernels) on the region's stream. i: index of the step in
// its block (selects the timing-event pair when a kernel is timed).
constexpr int ACT_EVERY = 32;  // eager blocks rebuild the list at most this often

// Bounded region: rebuild the list of advancing points for the next K steps.
void issue_act(semipar_region* r, int K) {
  if (!r->act) return;
  const int n = (int)r->n;
  const int nb = blocks(n);
  const int32_t* start = r->hist ? r->hstart : nullptr;
  k_act_count<<<nb, NT, 0, r->stream>>>(n, r->fstep, start, K - 1, r->actblk, r->ctrl);
  k_act_scan<<<1, 1024, 0, r->stream>>>(nb, r->actblk, r->ctrl);
  k_act_write<<<nb, NT, 0, r->stream>>>(n, r->fstep, start, K - 1, r->actblk, r->act, r->ctrl);
}

void issue_step(semipar_region* r, bool intercommute, int i) {
  const int n = (int)r->n;
  const int nb = blocks(n);
  const int nbe = std::min(nb, POINT_GRID);  // grid of the per-point kernels
  hipStream_t s = r->stream;
  const bool frw = r->cosmology != SEMIPAR_FLAT;
  mark(r, SEMIPAR_K_EVOLVE, 2 * i);
  const int scr = intercommute ? r->screen : 0;
  launch_evolve(r, frw, scr, r->bounded, n, nbe);
  mark(r, SEMIPAR_K_EVOLVE, 2 * i + 1);
  if (intercommute) {
    mark(r, SEMIPAR_K_SCAN, 2 * i);
    k_scan<<<r->ntiles, 256, 0, s>>>(r->cnt, r->loc, r->tile_tot, r->ctrl);
    mark(r, SEMIPAR_K_SCAN, 2 * i + 1);
    mark(r, SEMIPAR_K_SCATTER, 2 * i);
    k_toff<<<1, 1024, 0, s>>>(r->tile_tot, r->ntiles, r->toff, r->ctrl);
    PencilAux* saux = r->split == SPLIT_PRE ? r->saux : nullptr;
    if (r->screen == 1)
      k_scatter<1><<<nbe, NT, 0, s>>>(n, r->ecell, r->cnt, r->loc, r->toff, r->ebox, r->sent,
                                      r->sbox, r->hc, r->rid, r->rcell, r->wlive, r->ctrl, saux,
                                      r->nxt, r->prv, r->act);
    else
      k_scatter<2><<<nbe, NT, 0, s>>>(n, r->ecell, r->cnt, r->loc, r->toff, r->ebox, r->sent,
                                      r->sbox, r->hc, r->rid, r->rcell, r->wlive, r->ctrl, saux,
                                      r->nxt, r->prv, r->act);
    mark(r, SEMIPAR_K_SCATTER, 2 * i + 1);
    mark(r, SEMIPAR_K_SCREEN, 2 * i);
    launch_screen(r, n, nb);
    mark(r, SEMIPAR_K_SCREEN, 2 * i + 1);
    mark(r, SEMIPAR_K_CONFIRM, 2 * i);
    k_confirm<<<512, NT, 0, s>>>(r->X, r->nxt, r->id, r->P, r->cand, (int)r->cap_cand, r->ev,
                                 (int)r->cap_evt, r->ctrl);
    mark(r, SEMIPAR_K_CONFIRM, 2 * i + 1);
  }
  mark(r, SEMIPAR_K_RESOLVE, 2 * i);
  // one workgroup per group of sub-regions (their events never share an element)
  const int ngrp = r->rid ? std::max(1, std::min<int>(r->n_sub, RES_GROUPS)) : 1;
  k_resolve<<<ngrp, RESOLVE_NT, 0, s>>>(r->nxt, r->prv, r->ev, (int)r->cap_evt, (int)r->cap_cand,
                                     r->best, r->used, r->evs, r->log, r->log_cap, r->blkred, nbe,
                                     r->ctrl, r->rid, r->log_rid, r->lev, r->p_ic, r->seed,
                                     r->geoms, r->n_sub, r->rext,
                                     intercommute ? r->rcell : nullptr, r->rc_fixed_h);
  mark(r, SEMIPAR_K_RESOLVE, 2 * i + 1);
}

int read_ctrl(semipar_region* r);

// A batch can be evolved by persistent workgroups when every sub-region is small, the
// call runs to the regions' own stop (no loop removal, no time limit) and no kernel is
// being timed.
bool persistent_ok(const semipar_region* r, const semipar_evolve_params* p) {
  if (r->n_sub <= 0 || !r->rid || !p->intercommute || p->loop_every != 0 ||
      p->timed_kernel >= 0 || !std::isinf(p->t_end) || r->removed)
    return false;
  for (int q = 0; q < r->n_sub; ++q)
    if (r->sub_off[q + 1] - r->sub_off[q] > PB_MAXP) return false;
  return true;
}

// Evolve every sub-region of a batch of small regions to its own stop in one launch of
// persistent workgroups (k_region_block). A step with more crossings than a workgroup
// holds, or a full event log, gives SEMIPAR_E_OVERFLOW and leaves the region unusable:
// it is then run again from its surfaces on the step kernels.
int evolve_persistent(semipar_region* r, const semipar_evolve_params* p,
                      semipar_evolve_stats* st, const Ctrl& before, int32_t step_limit) {
  const int ns = r->n_sub;
  if (!r->dsub_off) {
    HIPCHK(dalloc(&r->dsub_off, (size_t)ns + 1));
    HIPCHK(dalloc(&r->pb_head, 1));
    HIPCHK(hipMemcpyAsync(r->dsub_off, r->sub_off.data(), sizeof(int64_t) * ((size_t)ns + 1),
                          hipMemcpyHostToDevice, r->stream));
  }
  // room for many more events than such regions have (about one per six points over a
  // whole run); the launch stops cleanly if the log fills anyway
  RCCHK(ensure_log(r, r->ctrl_h->log_n + 8 * r->n + 65536));
  drop_graph(r);
  HIPCHK(hipMemsetAsync(r->pb_head, 0, sizeof(int32_t), r->stream));
  HIPCHK(hipEventRecord(r->ev0, r->stream));
  const int grid = std::min(ns, PB_GRID);
  if (r->cosmology != SEMIPAR_FLAT)
    k_region_block<true><<<grid, PB_NT, 0, r->stream>>>(
        r->X, r->nxt, r->prv, r->id, r->fstep, r->face, r->frz, r->lev, r->geoms, r->dsub_off,
        ns, r->pb_head, r->P, r->hcoef, before.step, step_limit, r->p_ic, r->seed, r->log,
        r->log_rid, r->log_cap, r->ctrl);
  else
    k_region_block<false><<<grid, PB_NT, 0, r->stream>>>(
        r->X, r->nxt, r->prv, r->id, r->fstep, r->face, r->frz, r->lev, r->geoms, r->dsub_off,
        ns, r->pb_head, r->P, r->hcoef, before.step, step_limit, r->p_ic, r->seed, r->log,
        r->log_rid, r->log_cap, r->ctrl);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(r->ev1, r->stream));
  RCCHK(read_ctrl(r));
  Ctrl c = *r->ctrl_h;
  if (c.err & 64) {
    r->broken = true;
    spi::set_error("region_evolve: a step of a persistent region held more crossings than its "
                   "workgroup keeps, or the event log filled; run the regions on the step kernels");
    return SEMIPAR_E_OVERFLOW;
  }
  const int32_t fs = std::max(c.pb_step, before.step);
  c.steps_taken += fs - before.step;
  c.step = fs;
  c.pb_step = 0;
  c.done = 1;
  *r->ctrl_h = c;
  HIPCHK(hipMemcpyAsync(r->ctrl, r->ctrl_h, sizeof(Ctrl), hipMemcpyHostToDevice, r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  if (st) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r->ev0, r->ev1);
    st->steps = fs - before.step;
    st->point_steps = c.point_steps - before.point_steps;
    st->candidates = c.cand_total - before.cand_total;
    st->confirmed = c.conf_total - before.conf_total;
    st->accepted = c.acc_total - before.acc_total;
    st->passed = c.pass_total - before.pass_total;
    st->final_step = fs;
    st->done = 1;
    st->elapsed_ms = ms;
  }
  return SEMIPAR_OK;
}

int read_ctrl(semipar_region* r) {
  HIPCHK(hipMemcpyAsync(r->ctrl_h, r->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  return SEMIPAR_OK;
}

__global__ void k_clear_defer(Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->defer = 0;
    ctrl->done = 0;
  }
}

// Per-point stop state the kernels read: always for a bounded region, and for a
// whole-volume region once a loop has been removed from it.
const int32_t* stop_state(const semipar_region* r) {
  return (r->bounded || r->removed) ? r->fstep : nullptr;
}

int loop_setup(semipar_region* r) {
  if (r->lab[0]) return SEMIPAR_OK;
  const int64_t cap = std::max<int64_t>(r->cap, 1);
  if (!r->frz) HIPCHK(dalloc(&r->frz, cap));
  for (int i = 0; i < 2; ++i) {
    HIPCHK(dalloc(&r->lab[i], cap));
    HIPCHK(dalloc(&r->lptr[i], cap));
  }
  HIPCHK(dalloc(&r->lcnt, cap));
  HIPCHK(dalloc(&r->levm, cap));
  HIPCHK(dalloc(&r->lbad, cap));
  HIPCHK(dalloc(&r->lidx, cap));
  HIPCHK(dalloc(&r->lrep, cap));
  HIPCHK(dalloc(&r->lctr, 2));
  HIPCHK(hipHostMalloc((void**)&r->lctr_h, 2 * sizeof(int32_t), hipHostMallocDefault));
  return SEMIPAR_OK;
}

int grow_loop_log(semipar_region* r, int64_t need) {
  if (r->llog_cap >= need) return SEMIPAR_OK;
  const int64_t nc = std::max<int64_t>(need, std::max<int64_t>(2 * r->llog_cap, 1024));
  semipar_loop* nl = nullptr;
  int32_t* nr = nullptr;
  HIPCHK(dalloc(&nl, nc));
  HIPCHK(dalloc(&nr, nc));
  if (r->llog_n > 0) {
    HIPCHK(hipMemcpyAsync(nl, r->llog, sizeof(semipar_loop) * r->llog_n, hipMemcpyDeviceToDevice,
                          r->stream));
    HIPCHK(hipMemcpyAsync(nr, r->llog_rid, sizeof(int32_t) * r->llog_n, hipMemcpyDeviceToDevice,
                          r->stream));
  }
  HIPCHK(hipStreamSynchronize(r->stream));
  if (r->llog) r->retired.push_back(r->llog);
  if (r->llog_rid) r->retired.push_back(r->llog_rid);
  r->llog = nl;
  r->llog_rid = nr;
  r->llog_cap = nc;
  return SEMIPAR_OK;
}

// Loop record and removal at the start of step s (between steps, never inside a
// captured graph). Adds the loops and points removed to *nl, *np.
int loop_check(semipar_region* r, int32_t s, int64_t* nl, int64_t* np) {
  RCCHK(loop_setup(r));
  const int n = (int)r->n;
  const int nb = blocks(n);
  hipStream_t st = r->stream;
  k_fill_i32<<<1, NT, 0, st>>>(r->lctr, 2, 0);
  k_loop_init<<<nb, NT, 0, st>>>(n, r->nxt, r->fstep, r->lab[0], r->lptr[0], r->lcnt, r->levm,
                                 r->lbad);
  int c = 0;
  for (int64_t span = 1; span < n; span <<= 1) {
    k_loop_jump<<<nb, NT, 0, st>>>(n, r->lab[c], r->lptr[c], r->lab[c ^ 1], r->lptr[c ^ 1]);
    c ^= 1;
  }
  k_loop_gather<<<nb, NT, 0, st>>>(n, s, r->X, r->lab[c], r->lev, r->box, r->lcnt, r->levm,
                                   r->lbad);
  k_loop_decide<<<nb, NT, 0, st>>>(n, s, r->lab[c], r->lcnt, r->levm, r->lbad, r->lidx, r->lrep,
                                   r->lctr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(r->lctr_h, r->lctr, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const int32_t loops = r->lctr_h[0], pts = r->lctr_h[1];
  if (loops == 0) return SEMIPAR_OK;
  if (r->lacc_cap < loops) {
    if (r->lacc) r->retired.push_back(r->lacc);
    r->lacc = nullptr;
    r->lacc_cap = 0;
    const int64_t want = std::max<int64_t>(loops, 256);
    HIPCHK(dalloc(&r->lacc, 4 * want));
    r->lacc_cap = want;
  }
  RCCHK(grow_loop_log(r, r->llog_n + loops));
  HIPCHK(hipMemsetAsync(r->lacc, 0, sizeof(double) * 4 * (size_t)loops, st));
  k_loop_apply<<<nb, NT, 0, st>>>(n, s, r->X, r->lab[c], r->lidx, r->nxt, r->prv, r->id, r->box,
                                  r->lacc, r->frz, r->fstep, r->face, r->ecell);
  k_loop_final<<<blocks(loops), NT, 0, st>>>(loops, s, r->X, r->lrep, r->lcnt, r->id, r->lacc,
                                             r->rid, r->llog + r->llog_n,
                                             r->llog_rid + r->llog_n);
  HIPCHK(hipGetLastError());
  r->llog_n += loops;
  *nl += loops;
  *np += pts;
  if (!r->removed) {
    // launches captured so far pass no stop state to whole-volume kernels
    r->removed = true;
    drop_graph(r);
  }
  return SEMIPAR_OK;
}

}  // namespace

extern "C" {

const char* semipar_strerror(int code) {
  switch (code) {
    case SEMIPAR_OK: return "ok";
    case SEMIPAR_E_ARG: return "invalid argument";
    case SEMIPAR_E_SURFACE: return "inconsistent surface (duplicate id, dangling link, mixed slices)";
    case SEMIPAR_E_OOM: return "out of memory";
    case SEMIPAR_E_HIP: return "HIP runtime error";
    case SEMIPAR_E_OVERFLOW: return "per-step buffer overflow";
    case SEMIPAR_E_STATE: return "call out of order";
    default: return "unknown error";
  }
}

const char* semipar_last_error(void) { return g_last_error; }

const char* semipar_version(void) {
  return "libsemipar 0.1 gfx950 " __VERSION__;
}

void region_destroy(semipar_region* r) {
  if (!r) return;
  drop_graph(r);
  free_step_buffers(r);
  for (void* q : r->retired) dfree(q);
  for (int s = 0; s < 3; ++s)
    dfree(r->X.p[s]);
  dfree(r->nxt);
  dfree(r->prv);
  dfree(r->id);
  dfree(r->blkred);
  dfree(r->geoms);
  dfree(r->rid);
  dfree(r->fstep);
  dfree(r->face);
  dfree(r->wlive);
  dfree(r->frz);
  dfree(r->ctrl);
  dfree(r->log);
  dfree(r->log_rid);
  dfree(r->rcell);
  dfree(r->rext);
  dfree(r->lev);
  dfree(r->dsub_off);
  dfree(r->pb_head);
  for (int i = 0; i < 2; ++i) {
    dfree(r->lab[i]);
    dfree(r->lptr[i]);
  }
  dfree(r->lcnt);
  dfree(r->levm);
  dfree(r->lbad);
  dfree(r->lidx);
  dfree(r->lrep);
  dfree(r->lctr);
  dfree(r->lacc);
  dfree(r->llog);
  dfree(r->llog_rid);
  dfree(r->act);
  dfree(r->actblk);
  dfree(r->hgsl);
  dfree(r->hgnx);
  dfree(r->hstart);
  dfree(r->hsname);
  dfree(r->htok);
  if (r->lctr_h) (void)hipHostFree(r->lctr_h);
  if (r->ctrl_h) (void)hipHostFree(r->ctrl_h);
  if (r->ev0) (void)hipEventDestroy(r->ev0);
  if (r->ev1) (void)hipEventDestroy(r->ev1);
  for (hipEvent_t e : r->tev) (void)hipEventDestroy(e);
  if (r->own_stream && r->stream) (void)hipStreamDestroy(r->stream);
  delete r;
  (void)hipGetLastError();  // a failed release is not reported by later launches
}

int region_init_from_surfaces(const semipar_region_desc* d, const semipar_surface* in, int n_in,
                              semipar_region** out) {
  spi::begin_call();
  if (!out) return SEMIPAR_E_ARG;
  *out = nullptr;
  if (!d || n_in < 0 || (n_in > 0 && !in)) return SEMIPAR_E_ARG;
  if (!(d->box > 0.0) || d->cosmology < 0 || d->cosmology > 2 || d->capacity < 0)
    return SEMIPAR_E_ARG;
  if (d->bounded && d->n_sub == 0 && !(d->inv2g > 0.0)) return SEMIPAR_E_ARG;
  if (d->n_sub < 0 || (d->n_sub > 0 && (!d->bounded || !d->sub || d->n_sub != n_in)))
    return SEMIPAR_E_ARG;
  for (int i = 0; i < d->n_sub; ++i)
    if (!(d->sub[i].inv2g > 0.0)) return SEMIPAR_E_ARG;
  int64_t total = 0;
  for (int i = 0; i < n_in; ++i) {
    if (in[i].n < 0 || (in[i].n > 0 && !in[i].recs)) return SEMIPAR_E_ARG;
    if (in[i].mem != SEMIPAR_MEM_HOST && in[i].mem != SEMIPAR_MEM_DEVICE) return SEMIPAR_E_ARG;
    total += in[i].n;
  }
  if (total >= (int64_t)1 << 30 || d->capacity >= (int64_t)1 << 30) return SEMIPAR_E_ARG;
  if (d->capacity > 0 && d->capacity < total) return SEMIPAR_E_ARG;
  semipar_region* r = new (std::nothrow) semipar_region();
  if (!r) return SEMIPAR_E_OOM;
  r->n = total;
  r->cap = d->capacity > 0 ? d->capacity : total;
  r->cosmology = d->cosmology;
  r->hcoef = d->cosmology == SEMIPAR_MATTER ? 2.0 : (d->cosmology == SEMIPAR_RADIATION ? 1.0 : 0.0);
  r->box = d->box;
  r->bounded = d->bounded != 0;
  if (r->bounded) {
    for (int i = 0; i < 4; ++i) {
      r->geom.V[i] = d->origin[i];
      r->geom.idx[i] = d->idx[i];
    }
    r->geom.inv2g = d->inv2g;
    r->geom.sqrt3 = std::sqrt(3.0);
  }
  {
    int ex = 0;
    const double mant = std::frexp(d->box, &ex);
    r->P.box = d->box;
    r->P.pow2 = mant == 0.5 ? 1 : 0;
    r->P.inv = r->P.pow2 ? std::ldexp(1.0, 1 - ex) : 1.0 / d->box;
  }
  r->stream = (hipStream_t)d->stream;
  int rc = SEMIPAR_OK;
  auto fail = [&](int code) {
    region_destroy(r);
    return code;
  };
  if (!r->stream) {
    // The legacy null stream cannot be captured into a graph: use a blocking stream of
    // our own (default priority), which orders itself against the null stream.
    if (hipStreamCreate(&r->stream) != hipSuccess) return fail(SEMIPAR_E_HIP);
    r->own_stream = true;
  }
  const int64_t cap = std::max<int64_t>(r->cap, 1);
  for (int s = 0; s < 3; ++s)
    if (dalloc(&r->X.p[s], cap) != hipSuccess) return fail(oom(__LINE__));
  if (dalloc(&r->nxt, cap) != hipSuccess || dalloc(&r->prv, cap) != hipSuccess ||
      dalloc(&r->id, cap) != hipSuccess || dalloc(&r->ctrl, 1) != hipSuccess ||
      dalloc(&r->blkred, 4 * (size_t)blocks(cap)) != hipSuccess ||
      dalloc(&r->fstep, cap) != hipSuccess || dalloc(&r->face, cap) != hipSuccess ||
      dalloc(&r->lev, cap) != hipSuccess || dalloc(&r->wlive, (cap + 63) / 64) != hipSuccess ||
      (d->bounded && dalloc(&r->frz, cap) != hipSuccess) ||
      (d->bounded && (dalloc(&r->act, cap) != hipSuccess ||
                      dalloc(&r->actblk, (size_t)blocks(cap)) != hipSuccess)))
    return fail(oom(__LINE__));
  if (hipHostMalloc((void**)&r->ctrl_h, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess)
    return fail(oom(__LINE__));
  // Every copy and fill goes on the region's stream: a null-stream operation waits for
  // all streams, and invalidates a graph capture in progress on any other thread (a
  // batch on another lane of the scheduler).
  if (hipMemsetAsync(r->wlive, 1, (size_t)(cap + 63) / 64, r->stream) != hipSuccess)
    return fail(SEMIPAR_E_HIP);
  if (d->n_sub > 0) {
    // batch: per-point sub-region ids (surface order) and the geometry table
    r->n_sub = d->n_sub;
    std::vector<RegionGeom> hg((size_t)d->n_sub);
    for (int i = 0; i < d->n_sub; ++i) {
      for (int q = 0; q < 4; ++q) {
        hg[i].V[q] = d->sub[i].origin[q];
        hg[i].idx[q] = d->sub[i].idx[q];
      }
      hg[i].inv2g = d->sub[i].inv2g;
      hg[i].sqrt3 = std::sqrt(3.0);
    }
    int64_t off = 0;
    r->sub_off.assign((size_t)n_in + 1, 0);
    for (int i = 0; i < n_in; ++i) {
      r->sub_off[i] = off;
      off += in[i].n;
    }
    r->sub_off[n_in] = off;
    if (dalloc(&r->geoms, d->n_sub) != hipSuccess || dalloc(&r->rid, cap) != hipSuccess ||
        dalloc(&r->rcell, d->n_sub) != hipSuccess ||
        dalloc(&r->rext, (size_t)d->n_sub * REXT_STRIDE) != hipSuccess)
      return fail(oom(__LINE__));
    if (hipMemsetAsync(r->rcell, 0, sizeof(RCell) * d->n_sub, r->stream) != hipSuccess ||
        hipMemsetAsync(r->rext, 0, sizeof(uint64_t) * d->n_sub * REXT_STRIDE, r->stream) !=
            hipSuccess ||
        hipMemcpyAsync(r->geoms, hg.data(), sizeof(RegionGeom) * d->n_sub, hipMemcpyHostToDevice,
                       r->stream) != hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess)  // hg is read before it goes
      return fail(SEMIPAR_E_HIP);
    if (total > 0) {
      // sub-region of each slot, filled on the device from the sub-region offsets
      int64_t* doff = nullptr;
      if (salloc(&doff, (size_t)n_in + 1, r->stream) != hipSuccess) return fail(oom(__LINE__));
      const bool ok =
          hipMemcpyAsync(doff, r->sub_off.data(), sizeof(int64_t) * ((size_t)n_in + 1),
                         hipMemcpyHostToDevice, r->stream) == hipSuccess;
      if (ok)
        k_fill_rid<<<blocks(total), NT, 0, r->stream>>>(r->rid, (int)total, doff, n_in);
      const bool ok2 = ok && hipGetLastError() == hipSuccess &&
                       hipStreamSynchronize(r->stream) == hipSuccess;
      sfree(doff, r->stream);
      if (!ok2) return fail(SEMIPAR_E_HIP);
    }
  }
  if (hipEventCreate(&r->ev0) != hipSuccess || hipEventCreate(&r->ev1) != hipSuccess)
    return fail(SEMIPAR_E_HIP);
  Ctrl c0{};
  c0.step = 1;
  c0.tmin_key = KEY_MAX;
  c0.n_points = total;
  c0.step_limit = 1;
  c0.done = 1;
  c0.ext_key = 0;
  c0.box = d->box;
  c0.grow = CELL_GROW;
  c0.tol = d->box * std::ldexp(1.0, -30);
  if (total > 0) {
    // gather all surfaces into one device record array
    semipar_point_rec* drec = nullptr;
    if (salloc(&drec, total, r->stream) != hipSuccess) return fail(oom(__LINE__));
    int64_t off = 0;
    for (int i = 0; i < n_in; ++i) {
      if (in[i].n == 0) continue;
      const hipMemcpyKind kind =
          in[i].mem == SEMIPAR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
      if (hipMemcpyAsync(drec + off, in[i].recs, sizeof(semipar_point_rec) * in[i].n, kind,
                         r->stream) != hipSuccess) {
        sfree(drec, r->stream);
        return fail(SEMIPAR_E_HIP);
      }
      off += in[i].n;
    }
    semipar_point_rec rec0;
    if (hipMemcpyAsync(&rec0, drec, sizeof(rec0), hipMemcpyDeviceToHost, r->stream) != hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess) {
      sfree(drec, r->stream);
      return fail(SEMIPAR_E_HIP);
    }
    c0.step = rec0.step;
    r->step0 = rec0.step;
    const uint64_t hcap = next_pow2(2 * (uint64_t)total);
    int64_t* hkey = nullptr;
    int32_t* hval = nullptr;
    if (salloc(&hkey, hcap, r->stream) != hipSuccess ||
        salloc(&hval, hcap, r->stream) != hipSuccess) {
      sfree(drec, r->stream);
      sfree(hkey, r->stream);
      sfree(hval, r->stream);
      return fail(oom(__LINE__));
    }
    const int n = (int)total;
    rc = SEMIPAR_OK;
    if (hipMemcpyAsync(r->ctrl, &c0, sizeof(Ctrl), hipMemcpyHostToDevice, r->stream) != hipSuccess)
      rc = SEMIPAR_E_HIP;
    if (rc == SEMIPAR_OK) {
      k_fill_i64<<<blocks((int64_t)hcap), NT, 0, r->stream>>>(hkey, hcap, ID_EMPTY);
      k_init_insert<<<blocks(n), NT, 0, r->stream>>>(drec, n, hkey, hval, (uint32_t)(hcap - 1),
                                                     r->ctrl);
      k_init_links<<<blocks(n), NT, 0, r->stream>>>(drec, n, hkey, hval, (uint32_t)(hcap - 1), r->X,
                                                    r->nxt, r->prv, r->id, r->bounded ? 1 : 0,
                                                    r->fstep, r->face, r->lev, r->rid, r->ctrl);
      k_init_check<<<blocks(n), NT, 0, r->stream>>>(r->X, n, r->nxt, r->prv, r->P, c0.step,
                                                    r->ctrl);
      if (hipError_t e_ = hipGetLastError(); e_ != hipSuccess) rc = hip_fail(e_, "launch", __LINE__);
    }
    if (rc == SEMIPAR_OK && read_ctrl(r) != SEMIPAR_OK) rc = SEMIPAR_E_HIP;
    sfree(drec, r->stream);
    sfree(hkey, r->stream);
    sfree(hval, r->stream);
    if (rc != SEMIPAR_OK) return fail(rc);
    if (r->ctrl_h->err != 0) return fail(SEMIPAR_E_SURFACE);
    r->ext0 = from_key(r->ctrl_h->ext_key);
  } else {
    if (hipMemcpyAsync(r->ctrl, &c0, sizeof(Ctrl), hipMemcpyHostToDevice, r->stream) !=
            hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess)
      return fail(SEMIPAR_E_HIP);
    *r->ctrl_h = c0;
  }
  if (ensure_log(r, 1 << 16) != SEMIPAR_OK) return fail(oom(__LINE__));
  *out = r;
  return SEMIPAR_OK;
}

int region_evolve(semipar_region* r, const semipar_evolve_params* p, semipar_evolve_stats* st) {
  spi::begin_call();
  if (!r || !p || p->max_steps < 0 || p->loop_every < 0) return SEMIPAR_E_ARG;
  if (p->screen != SEMIPAR_SCREEN_F64 && p->screen != SEMIPAR_SCREEN_F32) return SEMIPAR_E_ARG;
  if (r->hist && p->loop_every != 0) return SEMIPAR_E_ARG;
  // a hand-off batch passes every crossing through (links never change)
  const double p_ic = r->hist ? 0.0 : (p->p == 0.0 ? 1.0 : p->p);
  if (!(p_ic >= 0.0 && p_ic <= 1.0) || (!r->hist && p_ic == 0.0)) return SEMIPAR_E_ARG;
  if (!(p->cell_factor == 0.0 || (p->cell_factor >= 1.0 && p->cell_factor <= 4.0)))
    return SEMIPAR_E_ARG;
  if (r->broken) return SEMIPAR_E_STATE;
  semipar_evolve_stats zero{};
  if (st) *st = zero;
  if (r->n == 0 || p->max_steps == 0) {
    if (st) {
      st->final_step = r->ctrl_h->step;
      st->done = 1;
    }
    return SEMIPAR_OK;
  }
  int rc = configure(r, p);
  if (rc != SEMIPAR_OK) return rc;
  RCCHK(read_ctrl(r));
  const Ctrl before = *r->ctrl_h;
  const int64_t lim64 = (int64_t)before.step + p->max_steps;
  const int32_t step_limit = (int32_t)std::min<int64_t>(lim64, INT32_MAX - 1);
  const int n = (int)r->n;
  const bool ic = p->intercommute != 0;
  const int K = p->steps_per_sync > 0 ? p->steps_per_sync : 32;
  {
    const int sp_ = p->screen_split;
    const int split = sp_ == 1 ? 1 : (sp_ == SPLIT_PRE ? SPLIT_PRE : N_PENCIL);
    if (split != r->split) drop_graph(r);
    r->split = split;
    if (split == SPLIT_PRE && !r->saux) {
      drop_graph(r);
      if (dalloc(&r->saux, (size_t)std::max<int64_t>(r->cap, 1)) != hipSuccess)
        return oom(__LINE__);
    }
    if (p_ic != r->p_ic || p->seed != r->seed) drop_graph(r);
    r->p_ic = p_ic;
    r->seed = p->seed;
  }
  if (p->persistent && !r->hist && persistent_ok(r, p))
    return evolve_persistent(r, p, st, before, step_limit);
  r->timed = (p->timed_kernel >= 0 && p->timed_kernel <= SEMIPAR_K_RESOLVE) ? p->timed_kernel : -1;
  if (r->timed >= 0) {
    rc = ensure_timing_events(r, K);
    if (rc != SEMIPAR_OK) return rc;
  }
  double tk_ms = 0.0;
  int64_t tk_n = 0;
  // Loop checks come before every step n with n - n0 a positive multiple of P: the
  // steps run in segments that end at the next such n (or at the call's limit).
  const int32_t P = p->loop_every;
  const int32_t s0 = r->step0;
  auto is_check = [&](int32_t s) {
    return P > 0 && s > s0 && ((int64_t)s - s0) % P == 0;
  };
  auto seg_limit = [&](int32_t s) -> int32_t {
    if (P <= 0) return step_limit;
    const int64_t c = (int64_t)s0 + (((int64_t)s - s0) / P + 1) * (int64_t)P;
    return (int32_t)std::min<int64_t>(c, step_limit);
  };
  int64_t n_loops = 0, n_lpts = 0;
  int32_t checked = INT32_MIN;
  HIPCHK(hipEventRecord(r->ev0, r->stream));
  if (is_check(before.step)) {
    RCCHK(loop_check(r, before.step, &n_loops, &n_lpts));
    checked = before.step;
  }
  k_begin_min<<<blocks(n), NT, 0, r->stream>>>(r->X, n, stop_state(r), r->blkred, r->ctrl);
  // grid of the first step: the caller's cell size (kept fixed), else 1.25 x the
  // initial element-size estimate, then adapted each step to the largest element (cell
  // edge = grow x the previous step's largest extent)
  const double grow = p->cell_factor > 0 ? p->cell_factor : CELL_GROW;
  Cells cells{};
  int set_cells = 0;
  if (p->cell_size > 0) {
    cells = choose_cells(r->box, p->cell_size, r->hc.tol);
    cells.fixed = 1;
    set_cells = 1;
    r->cells_set = true;
    r->cells_fixed = true;
  } else if (!r->cells_set || r->cells_fixed) {
    cells = choose_cells(r->box, r->ext0 > 0 ? 1.25 * r->ext0 : r->box, r->hc.tol);
    set_cells = 1;
    r->cells_set = true;
    r->cells_fixed = false;
  }
  k_begin_set<<<1, 1024, 0, r->stream>>>(r->ctrl, seg_limit(before.step), p->t_end, r->blkred,
                                         blocks(n), cells, set_cells, grow);
  if (r->rcell) {
    // batch: every sub-region starts with cells fitting the largest initial element
    // (or the fixed size), then follows its own elements
    const double fh = p->cell_size > 0 ? p->cell_size : 0.0;
    if (fh != r->rc_fixed_h) drop_graph(r);  // the per-step launch carries it
    r->rc_fixed_h = fh;
    const double h0 = p->cell_size > 0 ? p->cell_size : 1.25 * std::max(r->ext0, 1e-300);
    k_rcells<<<1, 1024, 0, r->stream>>>(r->geoms, r->n_sub, r->rext, r->rcell, h0, r->ctrl);
  }
  HIPCHK(hipGetLastError());
  for (;;) {
    rc = ensure_log(r, r->ctrl_h->log_n + 2 * r->cap_evt);
    if (rc != SEMIPAR_OK) return rc;
    if (r->hist) {
      // every point writes at most one token per step: room for a whole block
      rc = ensure_tokens(r, r->ctrl_h->tok_n + (int64_t)K * r->n);
      if (rc != SEMIPAR_OK) return rc;
    }
    const int64_t taken0 = r->ctrl_h->steps_taken;
    // HIP events recorded inside a captured graph cannot be timed: a timed call
    // issues its steps eagerly.
    if (p->use_graph && r->timed < 0) {
      if (!r->gexec || r->g_steps != K || r->g_timed != r->timed) {
        drop_graph(r);
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(r->stream, hipStreamCaptureModeThreadLocal));
        issue_act(r, K);
        for (int i = 0; i < K; ++i) issue_step(r, ic, i);
        HIPCHK(hipStreamEndCapture(r->stream, &g));
        HIPCHK(hipGraphInstantiate(&r->gexec, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        r->g_steps = K;
        r->g_timed = r->timed;
      }
      HIPCHK(hipGraphLaunch(r->gexec, r->stream));
      r->act_last = INT32_MIN;  // the graph rebuilds the list for its own block only
    } else {
      // eager blocks rebuild the list only when this block runs past the steps it covers
      // (at least ACT_EVERY of them), so that blocks of one step do not pay for it each step
      const int32_t s = r->ctrl_h->step;
      if (r->act && (int64_t)s + K - 1 > (int64_t)r->act_last) {
        const int H = std::max(K, ACT_EVERY);
        issue_act(r, H);
        r->act_last = s + H - 1;
      }
      for (int i = 0; i < K; ++i) issue_step(r, ic, i);
      HIPCHK(hipGetLastError());
    }
    RCCHK(read_ctrl(r));
    const Ctrl& c = *r->ctrl_h;
    if (r->timed >= 0) {
      const int64_t taken = c.steps_taken - taken0;
      for (int64_t i = 0; i < taken && i < K; ++i) {
        float e = 0.f;
        HIPCHK(hipEventElapsedTime(&e, r->tev[2 * i], r->tev[2 * i + 1]));
        tk_ms += e;
        tk_n += 1;
      }
    }
    if (c.defer) {
      // a per-step buffer was too small: the step was not taken; grow and retake it
      if (c.defer & 4) {
        rc = ensure_log(r, c.log_n + 4 * r->cap_evt);
        if (rc != SEMIPAR_OK) return rc;
      }
      if (c.defer & 3) {
        rc = grow_step_caps(r, c.defer);
        if (rc != SEMIPAR_OK) {
          r->broken = true;
          return rc;
        }
      }
      k_clear_defer<<<1, 64, 0, r->stream>>>(r->ctrl);
      HIPCHK(hipGetLastError());
      RCCHK(read_ctrl(r));
      continue;
    }
    if (c.done) {
      const int32_t s = c.step;
      if (is_check(s) && s < step_limit && s != checked) {
        // end of a segment: check, then the stop rule over the points still advancing
        RCCHK(loop_check(r, s, &n_loops, &n_lpts));
        checked = s;
        k_begin_min<<<blocks(n), NT, 0, r->stream>>>(r->X, n, stop_state(r), r->blkred, r->ctrl);
        k_begin_set<<<1, 1024, 0, r->stream>>>(r->ctrl, seg_limit(s), p->t_end, r->blkred,
                                               blocks(n), Cells{}, 0, grow);
        HIPCHK(hipGetLastError());
        RCCHK(read_ctrl(r));
        if (!r->ctrl_h->done) continue;
      }
      break;
    }
  }
  HIPCHK(hipEventRecord(r->ev1, r->stream));
  HIPCHK(hipEventSynchronize(r->ev1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, r->ev0, r->ev1));
  const Ctrl& a = *r->ctrl_h;
  if (r->hist && (a.err & HERR_MASK)) {
    r->broken = true;
    char msg[256];
    snprintf(msg, sizeof(msg),
             "hand-off batch: %s%s%s%s%s%s",
             (a.err & HERR_INPUT) ? "a diamond's input was never built; " : "",
             (a.err & HERR_START) ? "a start token for a diamond of another region; " : "",
             (a.err & HERR_SLICES) ? "the world sheet holds too few slices; " : "",
             (a.err & HERR_SELF) ? "a world line re-entered its region; " : "",
             (a.err & HERR_TOKENS) ? "token buffer overflow; " : "",
             (a.err & HERR_TIE) ? "a diamond's inputs have two homes of one layer; " : "");
    spi::set_error(msg);
    return (a.err & HERR_SLICES) ? SEMIPAR_E_OVERFLOW : SEMIPAR_E_STATE;
  }
  if (st) {
    st->steps = a.steps_taken - before.steps_taken;
    st->point_steps = a.point_steps - before.point_steps;
    st->candidates = a.cand_total - before.cand_total;
    st->confirmed = a.conf_total - before.conf_total;
    st->accepted = a.acc_total - before.acc_total;
    st->passed = a.pass_total - before.pass_total;
    st->large_elements = a.large_total - before.large_total;
    st->final_step = a.step;
    st->done = 1;
    st->elapsed_ms = ms;
    st->timed_kernel_ms = tk_ms;
    st->timed_kernel_launches = tk_n;
    st->loops = n_loops;
    st->loop_points = n_lpts;
    st->resolve_rounds = (int64_t)(uint32_t)(a.stamp - before.stamp);
  }
  return SEMIPAR_OK;
}

int region_emit_final_surfaces(semipar_region* r, semipar_point_rec* out[4], const int64_t cap[4],
                               int64_t n[4], int32_t mem) {
  spi::begin_call();
  if (!r || !n) return SEMIPAR_E_ARG;
  if (mem != SEMIPAR_MEM_HOST && mem != SEMIPAR_MEM_DEVICE) return SEMIPAR_E_ARG;
  for (int f = 0; f < 4; ++f) n[f] = 0;
  if (r->n == 0) return SEMIPAR_OK;
  RCCHK(read_ctrl(r));
  const int s = r->ctrl_h->step;
  const int nn = (int)r->n;
  const int nb = blocks(nn);
  const int32_t* fs = stop_state(r);
  int32_t *blkcnt = nullptr, *blkoff = nullptr, *tot = nullptr;
  semipar_point_rec* tmp = nullptr;
  int rc = SEMIPAR_OK;
  int32_t th[4] = {0, 0, 0, 0};
  if (dalloc(&blkcnt, 4 * (size_t)nb) != hipSuccess || dalloc(&blkoff, 4 * (size_t)nb) != hipSuccess ||
      dalloc(&tot, 4) != hipSuccess) {
    rc = oom(__LINE__);
  } else {
    k_emit_count<<<nb, NT, 0, r->stream>>>(nn, fs, r->frz, blkcnt);
    k_emit_scan<<<1, 1024, 0, r->stream>>>(blkcnt, nb, blkoff, tot);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(th, tot, sizeof(th), hipMemcpyDeviceToHost, r->stream) != hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess)
      rc = SEMIPAR_E_HIP;
  }
  if (rc == SEMIPAR_OK) {
    for (int f = 0; f < 4; ++f) n[f] = th[f];
    bool want = out != nullptr;
    for (int f = 0; f < 4 && want; ++f)
      if (n[f] > 0 && (!out[f] || !cap || cap[f] < n[f])) rc = SEMIPAR_E_ARG;
    if (want && rc == SEMIPAR_OK) {
      if (dalloc(&tmp, r->n) != hipSuccess) rc = oom(__LINE__);
      if (rc == SEMIPAR_OK) {
        k_emit_write<<<nb, NT, 0, r->stream>>>(r->X, nn, s, r->nxt, r->prv, r->id, fs, r->frz,
                                               blkoff, tot,
                                               r->bounded ? SEMIPAR_FLAG_ACTIVE : 0, tmp);
        if (hipError_t e_ = hipGetLastError(); e_ != hipSuccess) rc = hip_fail(e_, "launch", __LINE__);
        int64_t off = 0;
        const hipMemcpyKind kind =
            mem == SEMIPAR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        for (int f = 0; f < 4 && rc == SEMIPAR_OK; ++f) {
          if (n[f] > 0 &&
              hipMemcpyAsync(out[f], tmp + off, sizeof(semipar_point_rec) * n[f], kind,
                             r->stream) != hipSuccess)
            rc = SEMIPAR_E_HIP;
          off += n[f];
        }
        if (rc == SEMIPAR_OK && hipStreamSynchronize(r->stream) != hipSuccess) rc = SEMIPAR_E_HIP;
      }
    }
  }
  dfree(blkcnt);
  dfree(blkoff);
  dfree(tot);
  dfree(tmp);
  return rc;
}

int region_loops(const semipar_region* r, semipar_loop* buf, int64_t cap, int64_t* n) {
  spi::begin_call();
  if (!r || !n || cap < 0) return SEMIPAR_E_ARG;
  const int64_t total = r->llog_n;
  if (!buf) {
    *n = total;
    return SEMIPAR_OK;
  }
  std::vector<semipar_loop> all((size_t)total);
  if (total > 0) {
    HIPCHK(hipMemcpyAsync(all.data(), r->llog, sizeof(semipar_loop) * total, hipMemcpyDeviceToHost,
                          r->stream));
    HIPCHK(hipStreamSynchronize(r->stream));
  }
  std::sort(all.begin(), all.end(), [](const semipar_loop& a, const semipar_loop& b) {
    if (a.step != b.step) return a.step < b.step;
    return a.rep_id < b.rep_id;
  });
  const int64_t m = std::min(total, cap);
  if (m > 0) memcpy(buf, all.data(), sizeof(semipar_loop) * m);
  *n = m;
  return SEMIPAR_OK;
}

int region_events(const semipar_region* r, semipar_event* buf, int64_t cap, int64_t* n) {
  spi::begin_call();
  if (!r || !n || cap < 0) return SEMIPAR_E_ARG;
  semipar_region* rr = const_cast<semipar_region*>(r);
  RCCHK(read_ctrl(rr));
  const int64_t total = rr->ctrl_h->log_n;
  if (!buf) {
    *n = total;
    return SEMIPAR_OK;
  }
  std::vector<semipar_event> all((size_t)total);
  if (total > 0) {
    HIPCHK(hipMemcpyAsync(all.data(), rr->log, sizeof(semipar_event) * total, hipMemcpyDeviceToHost,
                          rr->stream));
    HIPCHK(hipStreamSynchronize(rr->stream));
  }
  // Listing order (the log is written in completion order within a step).
  std::sort(all.begin(), all.end(), [](const semipar_event& a, const semipar_event& b) {
    if (a.step != b.step) return a.step < b.step;
    if (a.t_star != b.t_star) return a.t_star < b.t_star;
    if (a.id_a != b.id_a) return a.id_a < b.id_a;
    return a.id_b < b.id_b;
  });
  const int64_t m = std::min(total, cap);
  if (m > 0) memcpy(buf, all.data(), sizeof(semipar_event) * m);
  *n = m;
  return SEMIPAR_OK;
}

int region_candidates(const semipar_region* r, int64_t* ids, int64_t cap, int64_t* n) {
  spi::begin_call();
  if (!r || !n || cap < 0) return SEMIPAR_E_ARG;
  semipar_region* rr = const_cast<semipar_region*>(r);
  if (r->n == 0 || !rr->cand) {
    *n = 0;
    return SEMIPAR_OK;
  }
  RCCHK(read_ctrl(rr));
  const int64_t total = std::min<int64_t>(rr->ctrl_h->last_cand, rr->cap_cand);
  if (!ids) {
    *n = total;
    return SEMIPAR_OK;
  }
  std::vector<int64_t> all(2 * (size_t)total);
  if (total > 0) {
    int64_t* d = nullptr;
    HIPCHK(dalloc(&d, 2 * (size_t)total));
    k_cand_ids<<<blocks(total), NT, 0, rr->stream>>>(rr->cand, total, rr->id, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(all.data(), d, sizeof(int64_t) * 2 * total, hipMemcpyDeviceToHost,
                         rr->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(rr->stream);
    dfree(d);
    if (e != hipSuccess) return hip_fail(e, "candidate copy", __LINE__);
  }
  std::vector<std::pair<int64_t, int64_t>> pr((size_t)total);
  for (int64_t i = 0; i < total; ++i) pr[i] = {all[2 * i], all[2 * i + 1]};
  std::sort(pr.begin(), pr.end());
  const int64_t m = std::min(total, cap);
  for (int64_t i = 0; i < m; ++i) {
    ids[2 * i] = pr[i].first;
    ids[2 * i + 1] = pr[i].second;
  }
  *n = m;
  return SEMIPAR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// internal calls for the scheduler and the cost model
// ---------------------------------------------------------------------------------
namespace spi {

int64_t region_points(const semipar_region* r) { return r ? r->n : 0; }

int region_prepare(semipar_region* r, const semipar_evolve_params* p) {
  if (!r || !p) return SEMIPAR_E_ARG;
  if (r->n == 0) return SEMIPAR_OK;
  RCCHK(configure(r, p));
  RCCHK(read_ctrl(r));
  if (p->loop_every > 0) {
    // loop buffers up front (hipFree inside a check would wait for other lanes' work)
    RCCHK(loop_setup(r));
    RCCHK(grow_loop_log(r, 1024));
    if (!r->lacc) {
      HIPCHK(dalloc(&r->lacc, 4 * 1024));
      r->lacc_cap = 1024;
    }
  }
  // the log size region_evolve asks for at its first block
  return ensure_log(r, r->ctrl_h->log_n + 2 * r->cap_evt);
}
hipStream_t region_stream(const semipar_region* r) { return r ? r->stream : nullptr; }

void set_error(const char* msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

void begin_call() {
  g_last_error[0] = 0;
  (void)hipGetLastError();
}

int batch_emit(semipar_region* r, semipar_point_rec* out, std::vector<int64_t>& cnt,
               const int64_t* out_base) {
  if (!r || r->n_sub <= 0 || !r->rid) return SEMIPAR_E_ARG;
  const int ns = r->n_sub;
  cnt.assign(4 * (size_t)ns, 0);
  if (r->n == 0) return SEMIPAR_OK;
  RCCHK(read_ctrl(r));
  const int s = r->ctrl_h->step;
  const int nn = (int)r->n;
  const int nb = blocks(nn);
  int32_t *blkcnt = nullptr, *blkoff = nullptr, *tot = nullptr, *pst = nullptr;
  int64_t* dst = nullptr;
  int rc = SEMIPAR_OK;
  std::vector<int32_t> hp(4 * (size_t)ns, 0);
  int32_t th[4] = {0, 0, 0, 0};
  hipStream_t st = r->stream;
  if (salloc(&blkcnt, 4 * (size_t)nb, st) != hipSuccess ||
      salloc(&blkoff, 4 * (size_t)nb, st) != hipSuccess || salloc(&tot, 4, st) != hipSuccess ||
      salloc(&pst, 4 * (size_t)ns, st) != hipSuccess || salloc(&dst, 4 * (size_t)ns, st) != hipSuccess)
    rc = oom(__LINE__);
  if (rc == SEMIPAR_OK) {
    k_emit_count<<<nb, NT, 0, r->stream>>>(nn, r->fstep, r->frz, blkcnt);
    k_emit_scan<<<1, 1024, 0, r->stream>>>(blkcnt, nb, blkoff, tot);
    k_emit_sub_start<<<nb, NT, 0, r->stream>>>(nn, r->fstep, r->frz, r->rid, blkoff, pst);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hp.data(), pst, sizeof(int32_t) * 4 * ns, hipMemcpyDeviceToHost,
                       r->stream) != hipSuccess ||
        hipMemcpyAsync(th, tot, sizeof(th), hipMemcpyDeviceToHost, r->stream) != hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess)
      rc = SEMIPAR_E_HIP;
  }
  if (rc == SEMIPAR_OK) {
    // per sub-region: stream counts from the prefixes at its first slot and at the
    // first slot of the next non-empty sub-region (the totals after the last one)
    std::vector<int64_t> hd(4 * (size_t)ns, 0);
    int next = -1;
    for (int q = ns - 1; q >= 0; --q) {
      const int64_t nq = r->sub_off[q + 1] - r->sub_off[q];
      if (nq == 0) continue;
      int64_t base = out_base ? out_base[q] : r->sub_off[q];
      for (int f = 0; f < 4; ++f) {
        const int64_t end = next >= 0 ? hp[4 * next + f] : th[f];
        cnt[4 * q + f] = end - hp[4 * q + f];
        hd[4 * q + f] = base;
        base += cnt[4 * q + f];
      }
      next = q;
    }
    if (hipMemcpyAsync(dst, hd.data(), sizeof(int64_t) * 4 * ns, hipMemcpyHostToDevice,
                       r->stream) != hipSuccess)
      rc = SEMIPAR_E_HIP;
    if (rc == SEMIPAR_OK) {
      k_emit_sub_write<<<nb, NT, 0, r->stream>>>(r->X, nn, s, r->nxt, r->prv, r->id, r->fstep,
                                                 r->frz, r->rid, blkoff, pst, dst, out);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(r->stream) != hipSuccess)
        rc = SEMIPAR_E_HIP;
    }
  }
  sfree(blkcnt, st);
  sfree(blkoff, st);
  sfree(tot, st);
  sfree(pst, st);
  sfree(dst, st);
  return rc;
}

int handoff_batch(const HandoffShared& sh, int lane, const int32_t* slot, const int32_t* start,
                  const std::vector<int64_t>& sub_off, const semipar_region_geom* geoms,
                  const int64_t* names, hipStream_t stream, semipar_region** out) {
  *out = nullptr;
  if (lane < 0) return SEMIPAR_E_ARG;
  int32_t* gmap = sh.gmap + (size_t)lane * (size_t)sh.n;
  const int ns = (int)sub_off.size() - 1;
  if (ns <= 0 || !sh.H || !sh.gmap) return SEMIPAR_E_ARG;
  const int64_t total = sub_off[ns];
  if (total <= 0 || total >= (int64_t)1 << 30) return SEMIPAR_E_ARG;
  semipar_region* r = new (std::nothrow) semipar_region();
  if (!r) return SEMIPAR_E_OOM;
  auto fail = [&](int code) {
    region_destroy(r);
    return code;
  };
  r->n = total;
  r->cap = total;
  r->cosmology = sh.cosmology;
  r->hcoef = sh.cosmology == SEMIPAR_MATTER ? 2.0 : (sh.cosmology == SEMIPAR_RADIATION ? 1.0 : 0.0);
  r->box = sh.box;
  r->bounded = true;
  r->hist = true;
  {
    int ex = 0;
    const double mant = std::frexp(sh.box, &ex);
    r->P.box = sh.box;
    r->P.pow2 = mant == 0.5 ? 1 : 0;
    r->P.inv = r->P.pow2 ? std::ldexp(1.0, 1 - ex) : 1.0 / sh.box;
  }
  r->stream = stream;
  if (!r->stream) {
    if (hipStreamCreate(&r->stream) != hipSuccess) return fail(SEMIPAR_E_HIP);
    r->own_stream = true;
  }
  const int64_t cap = total;
  const int n = (int)total;
  for (int q = 0; q < 3; ++q)
    if (dalloc(&r->X.p[q], cap) != hipSuccess) return fail(oom(__LINE__));
  if (dalloc(&r->nxt, cap) != hipSuccess || dalloc(&r->prv, cap) != hipSuccess ||
      dalloc(&r->id, cap) != hipSuccess || dalloc(&r->ctrl, 1) != hipSuccess ||
      dalloc(&r->blkred, 4 * (size_t)blocks(cap)) != hipSuccess ||
      dalloc(&r->fstep, cap) != hipSuccess || dalloc(&r->face, cap) != hipSuccess ||
      dalloc(&r->lev, cap) != hipSuccess || dalloc(&r->wlive, (cap + 63) / 64) != hipSuccess ||
      dalloc(&r->geoms, ns) != hipSuccess || dalloc(&r->rid, cap) != hipSuccess ||
      dalloc(&r->rcell, ns) != hipSuccess ||
      dalloc(&r->rext, (size_t)ns * REXT_STRIDE) != hipSuccess ||
      dalloc(&r->hgsl, cap) != hipSuccess || dalloc(&r->hgnx, cap) != hipSuccess ||
      dalloc(&r->hstart, cap) != hipSuccess || dalloc(&r->hsname, ns) != hipSuccess ||
      dalloc(&r->act, cap) != hipSuccess || dalloc(&r->actblk, (size_t)blocks(cap)) != hipSuccess)
    return fail(oom(__LINE__));
  if (hipHostMalloc((void**)&r->ctrl_h, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess)
    return fail(oom(__LINE__));
  r->n_sub = ns;
  r->sub_off = sub_off;
  std::vector<RegionGeom> hg((size_t)ns);
  for (int i = 0; i < ns; ++i) {
    for (int q = 0; q < 4; ++q) {
      hg[i].V[q] = geoms[i].origin[q];
      hg[i].idx[q] = geoms[i].idx[q];
    }
    hg[i].inv2g = geoms[i].inv2g;
    hg[i].sqrt3 = std::sqrt(3.0);
  }
  int32_t smin = INT32_MAX, smax = INT32_MIN;
  for (int64_t k = 0; k < total; ++k) {
    smin = std::min(smin, start[k]);
    smax = std::max(smax, start[k]);
  }
  if (smin - 1 < sh.s0 || smin < 1) return fail(SEMIPAR_E_ARG);
  r->step0 = smin;
  Ctrl c0{};
  c0.step = smin;
  c0.start_last = smax;
  c0.tmin_key = KEY_MAX;
  c0.n_points = total;
  c0.step_limit = smin;
  c0.done = 1;
  c0.box = sh.box;
  c0.grow = CELL_GROW;
  c0.tol = sh.box * std::ldexp(1.0, -30);
  HistCfg& h = r->hcfg;
  h.H = (double4*)sh.H;
  h.home = sh.home;
  h.n = sh.n;
  h.s0 = sh.s0;
  h.ns = sh.ns;
  for (int q = 0; q < 4; ++q) h.V[q] = sh.V[q];
  h.inv2g = sh.inv2g;
  h.sqrt3 = std::sqrt(3.0);
  h.K = sh.K;
  h.S_lo = sh.S_lo;
  h.S_hi = sh.S_hi;
  h.lut = sh.lut;
  h.sname = r->hsname;
  h.gnext = sh.gnext;
  h.gprev = sh.gprev;
  h.gsl = r->hgsl;
  h.gnx = r->hgnx;
  h.start = r->hstart;
  h.tok = nullptr;
  h.tok_cap = 0;
  int64_t* doff = nullptr;
  hipStream_t st = r->stream;
  int rc = SEMIPAR_OK;
  if (salloc(&doff, (size_t)ns + 1, st) != hipSuccess) return fail(oom(__LINE__));
  if (hipMemsetAsync(r->wlive, 1, (size_t)(cap + 63) / 64, st) != hipSuccess ||
      hipMemsetAsync(r->rcell, 0, sizeof(RCell) * ns, st) != hipSuccess ||
      hipMemsetAsync(r->rext, 0, sizeof(uint64_t) * ns * REXT_STRIDE, st) != hipSuccess ||
      hipMemcpyAsync(r->geoms, hg.data(), sizeof(RegionGeom) * ns, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(r->hgsl, slot, sizeof(int32_t) * total, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(r->hstart, start, sizeof(int32_t) * total, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(r->hsname, names, sizeof(int64_t) * ns, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(doff, sub_off.data(), sizeof(int64_t) * ((size_t)ns + 1),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(r->ctrl, &c0, sizeof(Ctrl), hipMemcpyHostToDevice, st) != hipSuccess)
    rc = SEMIPAR_E_HIP;
  for (int q = 0; q < 3 && rc == SEMIPAR_OK; ++q)
    if (hipMemsetAsync(r->X.p[q], 0, sizeof(double4) * cap, st) != hipSuccess) rc = SEMIPAR_E_HIP;
  if (rc == SEMIPAR_OK) {
    k_fill_rid<<<blocks(total), NT, 0, st>>>(r->rid, n, doff, ns);
    k_hand_init<<<blocks(total), NT, 0, st>>>(n, r->hgsl, r->hstart, sh.gnext, sh.gid, r->hgnx,
                                             r->id, r->fstep, r->face, r->lev, gmap);
    k_hand_links<<<blocks(total), NT, 0, st>>>(n, r->hgsl, r->hgnx, r->hstart, sh.gprev, gmap,
                                              r->rid, r->nxt, r->prv, r->hcfg, r->P, r->ctrl);
    k_hand_unmap<<<blocks(total), NT, 0, st>>>(n, r->hgsl, gmap);
    if (hipError_t e_ = hipGetLastError(); e_ != hipSuccess) rc = hip_fail(e_, "launch", __LINE__);
  }
  // the host arrays are read before the call returns
  if (rc == SEMIPAR_OK && read_ctrl(r) != SEMIPAR_OK) rc = SEMIPAR_E_HIP;
  sfree(doff, st);
  if (rc != SEMIPAR_OK) return fail(rc);
  r->ext0 = from_key(r->ctrl_h->ext_key);
  if (hipEventCreate(&r->ev0) != hipSuccess || hipEventCreate(&r->ev1) != hipSuccess)
    return fail(SEMIPAR_E_HIP);
  if (ensure_log(r, 1 << 16) != SEMIPAR_OK) return fail(oom(__LINE__));
  *out = r;
  return SEMIPAR_OK;
}

int handoff_ic(const HandoffShared& sh, const semipar_point_rec* drec, hipStream_t st,
               std::vector<HandTok>& tok) {
  tok.clear();
  if (sh.n <= 0 || sh.ns < 2 || sh.n >= (int64_t)1 << 31) return SEMIPAR_E_ARG;
  HistCfg h{};
  h.H = (double4*)sh.H;
  h.home = sh.home;
  h.n = sh.n;
  h.s0 = sh.s0;
  h.ns = sh.ns;
  for (int q = 0; q < 4; ++q) h.V[q] = sh.V[q];
  h.inv2g = sh.inv2g;
  h.sqrt3 = std::sqrt(3.0);
  h.K = sh.K;
  h.S_lo = sh.S_lo;
  h.S_hi = sh.S_hi;
  h.lut = sh.lut;
  h.gnext = sh.gnext;
  h.gprev = sh.gprev;
  HandTok* dt = nullptr;
  unsigned long long* dn = nullptr;
  int32_t* derr = nullptr;
  if (salloc(&dt, 2 * (size_t)sh.n, st) != hipSuccess || salloc(&dn, 1, st) != hipSuccess ||
      salloc(&derr, 1, st) != hipSuccess) {
    sfree(dt, st);
    sfree(dn, st);
    sfree(derr, st);
    return oom(__LINE__);
  }
  int rc = SEMIPAR_OK;
  unsigned long long nt = 0;
  int32_t herr = 0;
  const uint64_t cells = (uint64_t)sh.ns * (uint64_t)sh.n;
  if (hipMemsetAsync(dn, 0, sizeof(unsigned long long), st) != hipSuccess ||
      hipMemsetAsync(derr, 0, sizeof(int32_t), st) != hipSuccess)
    rc = SEMIPAR_E_HIP;
  if (rc == SEMIPAR_OK) {
    k_hist_fill<<<4096, NT, 0, st>>>((double4*)sh.H, sh.home, cells);
    k_hist_ic<<<blocks(sh.n), NT, 0, st>>>(drec, (int)sh.n, h, dt, dn, derr);
    if (hipError_t e_ = hipGetLastError(); e_ != hipSuccess) rc = hip_fail(e_, "launch", __LINE__);
  }
  if (rc == SEMIPAR_OK &&
      (hipMemcpyAsync(&nt, dn, sizeof(nt), hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipMemcpyAsync(&herr, derr, sizeof(herr), hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    rc = SEMIPAR_E_HIP;
  if (rc == SEMIPAR_OK && herr != 0) {
    spi::set_error("hand-off: initial surface vertices with two homes of one layer");
    rc = SEMIPAR_E_STATE;
  }
  if (rc == SEMIPAR_OK && nt > 0) {
    tok.resize((size_t)nt);
    if (hipMemcpyAsync(tok.data(), dt, sizeof(HandTok) * nt, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = SEMIPAR_E_HIP;
  }
  sfree(dt, st);
  sfree(dn, st);
  sfree(derr, st);
  return rc;
}

int handoff_tokens(semipar_region* r, std::vector<HandTok>& out) {
  out.clear();
  if (!r || !r->hist) return SEMIPAR_E_ARG;
  RCCHK(read_ctrl(r));
  const int64_t nt = std::min<int64_t>(r->ctrl_h->tok_n, r->hcfg.tok_cap);
  if (nt <= 0) return SEMIPAR_OK;
  out.resize((size_t)nt);
  HIPCHK(hipMemcpyAsync(out.data(), r->htok, sizeof(HandTok) * nt, hipMemcpyDeviceToHost,
                        r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  return SEMIPAR_OK;
}

int batch_stats(semipar_region* r, std::vector<int32_t>& steps, std::vector<int64_t>& psteps) {
  if (!r || !r->bounded) return SEMIPAR_E_ARG;
  const int ns = r->n_sub > 0 ? r->n_sub : 1;  // a lone bounded region is one sub-region
  steps.assign(ns, 0);
  psteps.assign(ns, 0);
  if (r->n == 0) return SEMIPAR_OK;
  RCCHK(read_ctrl(r));
  unsigned long long* ps = nullptr;
  int32_t* sm = nullptr;
  int rc = SEMIPAR_OK;
  if (salloc(&ps, ns, r->stream) != hipSuccess || salloc(&sm, ns, r->stream) != hipSuccess)
    rc = oom(__LINE__);
  if (rc == SEMIPAR_OK &&
      (hipMemsetAsync(ps, 0, sizeof(unsigned long long) * ns, r->stream) != hipSuccess ||
       hipMemsetAsync(sm, 0, sizeof(int32_t) * ns, r->stream) != hipSuccess))
    rc = SEMIPAR_E_HIP;
  if (rc == SEMIPAR_OK) {
    k_sub_stats<<<blocks(r->n), NT, 0, r->stream>>>((int)r->n, r->fstep, r->ctrl_h->step, r->step0,
                                                    r->rid, ps, sm, r->hstart);
    std::vector<unsigned long long> hps((size_t)ns);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hps.data(), ps, sizeof(unsigned long long) * ns, hipMemcpyDeviceToHost,
                       r->stream) != hipSuccess ||
        hipMemcpyAsync(steps.data(), sm, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, r->stream) !=
            hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess)
      rc = SEMIPAR_E_HIP;
    for (int q = 0; q < ns; ++q) psteps[q] = (int64_t)hps[q];
  }
  sfree(ps, r->stream);
  sfree(sm, r->stream);
  return rc;
}

int batch_events(semipar_region* r, std::vector<semipar_event>& ev, std::vector<int64_t>& off) {
  if (!r || r->n_sub <= 0 || !r->rid) return SEMIPAR_E_ARG;
  const int ns = r->n_sub;
  ev.clear();
  off.assign((size_t)ns + 1, 0);
  RCCHK(read_ctrl(r));
  const int64_t total = r->ctrl_h->log_n;
  if (total == 0) return SEMIPAR_OK;
  if (total >= INT32_MAX) return SEMIPAR_E_OVERFLOW;
  // the project's bitonic sort on the device (see k_ev_keys)
  int64_t npow = EVS_LDS;
  while (npow < total) npow <<= 1;
  EvKey* keys = nullptr;
  int32_t* cnt = nullptr;
  semipar_event* sorted = nullptr;
  int rc = SEMIPAR_OK;
  if (salloc(&keys, npow, r->stream) != hipSuccess ||
      salloc(&sorted, total, r->stream) != hipSuccess || salloc(&cnt, ns, r->stream) != hipSuccess)
    rc = oom(__LINE__);
  std::vector<int32_t> hc((size_t)ns, 0);
  if (rc == SEMIPAR_OK) {
    const int nbp = blocks(npow);
    hipStream_t st = r->stream;
    k_ev_keys<<<nbp, NT, 0, st>>>(r->log, r->log_rid, total, npow, keys);
    k_ev_bitonic_lds<<<(int)(npow / EVS_LDS), NT, 0, st>>>(keys, 2, EVS_LDS, r->log);
    for (int64_t kk = 2 * EVS_LDS; kk <= npow; kk <<= 1) {
      for (int64_t j = kk >> 1; j >= EVS_LDS; j >>= 1)
        k_ev_bitonic<<<nbp, NT, 0, st>>>(keys, npow, kk, j, r->log);
      k_ev_bitonic_lds<<<(int)(npow / EVS_LDS), NT, 0, st>>>(keys, kk, kk, r->log);
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemsetAsync(cnt, 0, sizeof(int32_t) * ns, st) != hipSuccess)
      rc = SEMIPAR_E_HIP;
    if (rc == SEMIPAR_OK) {
      k_ev_gather<<<blocks(total), NT, 0, st>>>(r->log, r->log_rid, keys, total, sorted, cnt);
      ev.resize((size_t)total);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(ev.data(), sorted, sizeof(semipar_event) * total, hipMemcpyDeviceToHost,
                         st) != hipSuccess ||
          hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        rc = SEMIPAR_E_HIP;
    }
  }
  for (int q = 0; q < ns; ++q) off[q + 1] = off[q] + hc[q];
  sfree(keys, r->stream);
  sfree(sorted, r->stream);
  sfree(cnt, r->stream);
  if (rc != SEMIPAR_OK) ev.clear();
  return rc;
}

int batch_loops(semipar_region* r, std::vector<semipar_loop>& lp, std::vector<int64_t>& off) {
  if (!r || r->n_sub <= 0) return SEMIPAR_E_ARG;
  const int ns = r->n_sub;
  lp.clear();
  off.assign((size_t)ns + 1, 0);
  const int64_t total = r->llog_n;
  if (total == 0) return SEMIPAR_OK;
  std::vector<semipar_loop> all((size_t)total);
  std::vector<int32_t> q((size_t)total);
  HIPCHK(hipMemcpyAsync(all.data(), r->llog, sizeof(semipar_loop) * total, hipMemcpyDeviceToHost,
                        r->stream));
  HIPCHK(hipMemcpyAsync(q.data(), r->llog_rid, sizeof(int32_t) * total, hipMemcpyDeviceToHost,
                        r->stream));
  HIPCHK(hipStreamSynchronize(r->stream));
  std::vector<int64_t> ord((size_t)total);
  for (int64_t i = 0; i < total; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    if (q[a] != q[b]) return q[a] < q[b];
    if (all[a].step != all[b].step) return all[a].step < all[b].step;
    return all[a].rep_id < all[b].rep_id;
  });
  lp.resize((size_t)total);
  for (int64_t i = 0; i < total; ++i) {
    lp[i] = all[ord[i]];
    off[q[ord[i]] + 1] += 1;
  }
  for (int i = 0; i < ns; ++i) off[i + 1] += off[i];
  return SEMIPAR_OK;
}

int batch_features(semipar_region* r, float* feat) {
  if (!r || r->n_sub <= 0 || !feat) return SEMIPAR_E_ARG;
  const int ns = r->n_sub;
  for (int64_t i = 0; i < 12 * (int64_t)ns; ++i) feat[i] = 0.f;
  if (r->n == 0) return SEMIPAR_OK;
  RCCHK(read_ctrl(r));
  double* acc = nullptr;
  int32_t* grid = nullptr;
  int64_t* np = nullptr;
  float* df = nullptr;
  int rc = SEMIPAR_OK;
  if (dalloc(&acc, FEAT_STRIDE * (size_t)ns) != hipSuccess ||
      dalloc(&grid, (size_t)FEAT_CELLS * ns) != hipSuccess || dalloc(&np, ns) != hipSuccess ||
      dalloc(&df, 12 * (size_t)ns) != hipSuccess)
    rc = oom(__LINE__);
  std::vector<int64_t> hn((size_t)ns);
  for (int q = 0; q < ns; ++q) hn[q] = r->sub_off[q + 1] - r->sub_off[q];
  if (rc == SEMIPAR_OK &&
      (hipMemsetAsync(acc, 0, sizeof(double) * FEAT_STRIDE * ns, r->stream) != hipSuccess ||
       hipMemsetAsync(grid, 0, sizeof(int32_t) * FEAT_CELLS * (size_t)ns, r->stream) != hipSuccess ||
       hipMemcpyAsync(np, hn.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, r->stream) !=
           hipSuccess))
    rc = SEMIPAR_E_HIP;
  if (rc == SEMIPAR_OK) {
    k_feat_points<<<blocks(r->n), NT, 0, r->stream>>>(r->X, (int)r->n, r->ctrl_h->step, r->nxt,
                                                      r->prv, r->rid, r->geoms, r->P, acc, grid);
    k_feat_final<<<ns, 256, 0, r->stream>>>(grid, acc, np, r->geoms, df);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(feat, df, sizeof(float) * 12 * ns, hipMemcpyDeviceToHost, r->stream) !=
            hipSuccess ||
        hipStreamSynchronize(r->stream) != hipSuccess)
      rc = SEMIPAR_E_HIP;
  }
  dfree(acc);
  dfree(grid);
  dfree(np);
  dfree(df);
  return rc;
}

int surface_features(const semipar_tiling* t, float* feat) {
  const int nr = t->n_regions;
  std::vector<int64_t> off((size_t)nr + 1, 0);
  std::vector<const semipar_point_rec*> ptr((size_t)nr, nullptr);
  for (int q = 0; q < nr; ++q) {
    const semipar_surface& sf = t->surfaces[q];
    if (sf.n > 0 && sf.mem != SEMIPAR_MEM_DEVICE) return SEMIPAR_E_ARG;
    off[q + 1] = off[q] + sf.n;
    ptr[q] = sf.recs;
  }
  for (int64_t i = 0; i < 12 * (int64_t)nr; ++i) feat[i] = 0.f;
  const int64_t total = off[nr];
  if (total == 0) return SEMIPAR_OK;
  if (total >= (int64_t)1 << 30) return SEMIPAR_E_ARG;
  const int n = (int)total;
  uint64_t hcap = 2;
  while (hcap < 2 * (uint64_t)total) hcap <<= 1;
  std::vector<RegionGeom> hg((size_t)nr);
  std::vector<int64_t> hn((size_t)nr);
  for (int q = 0; q < nr; ++q) {
    for (int i = 0; i < 4; ++i) {
      hg[q].V[i] = t->geoms[q].origin[i];
      hg[q].idx[i] = t->geoms[q].idx[i];
    }
    hg[q].inv2g = t->geoms[q].inv2g;
    hg[q].sqrt3 = std::sqrt(3.0);
    hn[q] = off[q + 1] - off[q];
  }
  sp::Period P{};
  {
    int ex = 0;
    const double mant = std::frexp(t->box, &ex);
    P.box = t->box;
    P.pow2 = mant == 0.5 ? 1 : 0;
    P.inv = P.pow2 ? std::ldexp(1.0, 1 - ex) : 1.0 / t->box;
  }
  hipStream_t st = (hipStream_t)t->stream;
  const semipar_point_rec** dsrf = nullptr;
  int64_t *doff = nullptr, *hkey = nullptr, *np = nullptr;
  int32_t *hval = nullptr, *err = nullptr, *grid = nullptr;
  RegionGeom* dgeo = nullptr;
  double* acc = nullptr;
  float* df = nullptr;
  int rc = SEMIPAR_OK;
  if (dalloc(&dsrf, (size_t)nr) != hipSuccess || dalloc(&doff, (size_t)nr + 1) != hipSuccess ||
      dalloc(&dgeo, (size_t)nr) != hipSuccess || dalloc(&np, (size_t)nr) != hipSuccess ||
      dalloc(&hkey, hcap) != hipSuccess || dalloc(&hval, hcap) != hipSuccess ||
      dalloc(&err, 1) != hipSuccess || dalloc(&acc, FEAT_STRIDE * (size_t)nr) != hipSuccess ||
      dalloc(&grid, (size_t)FEAT_CELLS * nr) != hipSuccess || dalloc(&df, 12 * (size_t)nr) != hipSuccess)
    rc = oom(__LINE__);
  int32_t herr = 0;
  if (rc == SEMIPAR_OK &&
      (hipMemcpyAsync(dsrf, ptr.data(), sizeof(void*) * nr, hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(doff, off.data(), sizeof(int64_t) * (nr + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(dgeo, hg.data(), sizeof(RegionGeom) * nr, hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(np, hn.data(), sizeof(int64_t) * nr, hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemsetAsync(err, 0, sizeof(int32_t), st) != hipSuccess ||
       hipMemsetAsync(acc, 0, sizeof(double) * FEAT_STRIDE * nr, st) != hipSuccess ||
       hipMemsetAsync(grid, 0, sizeof(int32_t) * FEAT_CELLS * (size_t)nr, st) != hipSuccess))
    rc = SEMIPAR_E_HIP;
  if (rc == SEMIPAR_OK) {
    const uint32_t hmask = (uint32_t)(hcap - 1);
    k_fill_i64<<<blocks((int64_t)hcap), NT, 0, st>>>(hkey, hcap, ID_EMPTY);
    k_featsurf_insert<<<blocks(n), NT, 0, st>>>(dsrf, doff, nr, n, hkey, hval, hmask, err);
    k_featsurf_points<<<blocks(n), NT, 0, st>>>(dsrf, doff, nr, n, hkey, hval, hmask, dgeo, P,
                                                acc, grid);
    k_feat_final<<<nr, 256, 0, st>>>(grid, acc, np, dgeo, df);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(feat, df, sizeof(float) * 12 * nr, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = SEMIPAR_E_HIP;
    else if (herr != 0)
      rc = SEMIPAR_E_SURFACE;
  }
  if (rc != SEMIPAR_OK)
    for (int64_t i = 0; i < 12 * (int64_t)nr; ++i) feat[i] = 0.f;
  dfree(dsrf);
  dfree(doff);
  dfree(dgeo);
  dfree(np);
  dfree(hkey);
  dfree(hval);
  dfree(err);
  dfree(acc);
  dfree(grid);
  dfree(df);
  return rc;
}

}  // namespace spi
