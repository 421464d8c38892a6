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

// Record an error message for semipar_last_error.
SP_HIDDEN void set_error(const char* msg);

// Start of an entry point: clears this thread's message and HIP's per-thread last
// error, so that a failure left by an earlier call (the caller's own, or a release
// whose result was ignored) is not taken for a failure of this call's launches.
SP_HIDDEN void begin_call();

}  // namespace spi
