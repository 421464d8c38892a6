// internal.h -- calls shared between the translation units of libsemipar (not exported).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "semipar.h"

#define SP_HIDDEN __attribute__((visibility("hidden")))

namespace spi {

// Allocate the step buffers and the event log that region_evolve with these
// parameters would allocate at its start (so that it frees nothing while running).
SP_HIDDEN int region_prepare(semipar_region* r, const semipar_evolve_params* p);

// Number of points and the stream of a region.
SP_HIDDEN int64_t region_points(const semipar_region* r);
SP_HIDDEN hipStream_t region_stream(const semipar_region* r);

// Batch of sub-regions (a region built with n_sub > 0), after region_evolve:
// records of every sub-region into dst (device memory): sub-region q occupies as many
// records as its input surface had points, from base[q] on (base == nullptr: from its
// first slot in the batch, so that dst holds r->n records), its four streams in order,
// each in slot order; cnt[4 q + f] = records of q on stream f. Temporaries are
// stream-ordered on the region's stream, so this waits for no other stream.
SP_HIDDEN int batch_emit(semipar_region* r, semipar_point_rec* dst, std::vector<int64_t>& cnt,
                         const int64_t* base = nullptr);

// Per sub-region: slices advanced by its furthest point and its point-steps.
SP_HIDDEN int batch_stats(semipar_region* r, std::vector<int32_t>& steps,
                          std::vector<int64_t>& psteps);

// Logged events grouped by sub-region (sub-region q's at off[q] .. off[q+1]), each
// group in listing order (step, t*, id_a, id_b).
SP_HIDDEN int batch_events(semipar_region* r, std::vector<semipar_event>& ev,
                           std::vector<int64_t>& off);

// Logged loops grouped by sub-region (sub-region q's at off[q] .. off[q+1]), each group
// sorted by (step, rep_id).
SP_HIDDEN int batch_loops(semipar_region* r, std::vector<semipar_loop>& lp,
                          std::vector<int64_t>& off);

// The 12 cost-model features of each sub-region's current surface (host, 12 n_sub).
SP_HIDDEN int batch_features(semipar_region* r, float* feat);

// The same features of every region of a tiling read in place from its surfaces, which
// must all be device memory (SEMIPAR_E_ARG otherwise, nothing launched): no region state
// is built, only an id table for the right neighbours (host, 12 n_regions).
SP_HIDDEN int surface_features(const semipar_tiling* t, float* feat);

// ---- hand-off tiling runs (schedule_handoff) ----------------------------------------

// A start token: point `slot` (of the volume's initial surface) builds its diamonds in
// region `region` from step `step` on, because its right neighbour's world line entered
// that region at slice step - 1.
struct HandTok {
  int32_t slot;
  int32_t step;
  int32_t region;
  int32_t pad;
};

// Device tables shared by every batch of a hand-off run (owned by its driver).
struct HandoffShared {
  double* H;        // world sheet: [slice - s0][slot] (x, y, z, t), t = NaN: not built
  int64_t* home;    // [slice - s0][slot]: name of each vertex's home region
  int64_t n;        // points of the volume
  int32_t s0, ns;   // first slice held, slices held
  double V[4];      // lattice origin (x, y, z, tau) shared by all regions
  double inv2g;     // 1 / (2 g)
  int32_t K, S_lo, S_hi;  // region names: layer S in [S_lo, S_hi], past vertex mod K
  const int32_t* lut;     // [(S - S_lo) K^3 + key] -> region index, -1: none
  const int32_t* gnext;   // per volume slot: right neighbour's slot
  const int32_t* gprev;   // per volume slot: left neighbour's slot
  const int64_t* gid;     // per volume slot: point id
  int32_t* gmap;          // per lane and volume slot, lanes x n: -1 between batches (the
                          // batch build's scratch; batches on different lanes overlap)
  int32_t cosmology;
  double box;
};

// A batch of hand-off sub-regions: sub-region q's points are slot[sub_off[q] ..
// sub_off[q+1]) (host, volume slots, ascending within a sub-region) with their start
// steps; geoms and names (host, n_sub each) are the sub-regions' geometry and names.
// The region evolves with region_evolve; crossings are logged and pass through.
// lane selects the batch build's scratch row of sh.gmap.
SP_HIDDEN int handoff_batch(const HandoffShared& sh, int lane, const int32_t* slot,
                            const int32_t* start, const std::vector<int64_t>& sub_off,
                            const semipar_region_geom* geoms, const int64_t* names,
                            hipStream_t stream, semipar_region** out);

// Fill the world sheet with t = NaN, write the initial surface's two slices (drec: n
// records in device memory, volume slot order) and return the start tokens they give
// (host copy, any order). Stream-ordered on st.
SP_HIDDEN int handoff_ic(const HandoffShared& sh, const semipar_point_rec* drec, hipStream_t st,
                         std::vector<HandTok>& tok);

// The start tokens a hand-off batch wrote for other regions (host copy, any order).
SP_HIDDEN int handoff_tokens(semipar_region* r, std::vector<HandTok>& out);

// Record an error message for semipar_last_error.
SP_HIDDEN void set_error(const char* msg);

// Start of an entry point: clears this thread's message and HIP's per-thread last
// error, so that a failure left by an earlier call (the caller's own, or a release
// whose result was ignored) is not taken for a failure of this call's launches.
SP_HIDDEN void begin_call();

}  // namespace spi
