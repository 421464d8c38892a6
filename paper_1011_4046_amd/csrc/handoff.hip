// handoff.hip -- a periodic spacetime tiling run region by region with hand-off.
//
// Paper, Section "Geometry": the 4-volume is cut into 4-cubes whose faces no signal
// crosses backwards, so each region can run alone given what its predecessors passed
// on; subsection "Initial conditions": the regions cut by the initial time take initial
// data where they are cut and predecessor output elsewhere (four families), later ones
// only predecessor output; subsection "Boundary conditions": a periodic volume is the
// same tiling with its successor lists wrapped. Section "Semi-parallel cosmic string
// simulation": a diamond is built by the region holding its earliest point, and a region
// passes the diamonds overlapping its final surfaces to its successors.
//
// On one GPU the whole world sheet fits in device memory, so nothing is copied between
// regions: every vertex is written once into a slice-major table by the region that
// builds it, and read from there by every later diamond that needs it. What a region
// does pass on is where its successors' work begins: when a vertex it builds is the first
// vertex of a world line in another region, that region's diamond of the line's left
// neighbour starts there (a start token). The manager here keeps the tokens per region
// and runs the regions layer by layer as launch batches (one set of step kernels over the
// points of many regions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <numeric>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "internal.h"
#include "semipar.h"

namespace {

int fail_msg(int code, const char* msg) {
  spi::set_error(msg);
  return code;
}

int hip_msg(hipError_t e, const char* what) {
  char msg[200];
  snprintf(msg, sizeof(msg), "schedule_handoff: %s failed: %s", what, hipGetErrorString(e));
  spi::set_error(msg);
  return SEMIPAR_E_HIP;
}

// Device buffers of one call, released on every return path.
struct Dev {
  std::vector<void*> bufs;
  hipStream_t own = nullptr;
  ~Dev() {
    for (void* p : bufs) (void)hipFree(p);
    if (own) (void)hipStreamDestroy(own);
    (void)hipGetLastError();
  }
  template <class T>
  hipError_t alloc(T** p, size_t count) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * std::max<size_t>(count, 1));
    if (e == hipSuccess) bufs.push_back(*p);
    return e;
  }
};

// Region name (S << 32 | key) from an index, as the step kernels name vertices.
int64_t region_name(const int32_t idx[4], int K) {
  const int64_t i0 = idx[0], i1 = idx[1], i2 = idx[2], i3 = idx[3];
  int64_t p[3] = {i0 + i1 - i2 - i3, i0 - i1 + i2 - i3, i0 - i1 - i2 + i3};
  for (int c = 0; c < 3; ++c) p[c] = ((p[c] % K) + K) % K;
  const int64_t S = i0 + i1 + i2 + i3;
  return (S << 32) | (int64_t)(uint32_t)((p[0] * K + p[1]) * K + p[2]);
}

}  // namespace

int schedule_handoff(const semipar_handoff* h, const semipar_sched_params* p,
                     semipar_sched_stats* st) {
  spi::begin_call();
  const auto t0 = std::chrono::steady_clock::now();
  if (!h || !p) return SEMIPAR_E_ARG;
  const int nr = h->n_regions;
  if (nr <= 0 || !h->geoms || !h->n_pred || !h->succ_off || !h->ic || h->n_points <= 0 ||
      !h->hist || h->hist_slices < 2 || !(h->box > 0.0) || h->cosmology < 0 ||
      h->cosmology > 2 || (h->ic_mem != SEMIPAR_MEM_HOST && h->ic_mem != SEMIPAR_MEM_DEVICE))
    return SEMIPAR_E_ARG;
  if (h->n_points >= ((int64_t)1 << 31) - 1 || h->hist_slices > INT32_MAX) return SEMIPAR_E_ARG;
  if (p->out || p->evolve.loop_every != 0 || p->batch_points < 0 ||
      (p->events && (!p->events_off || p->events_cap < 0)))
    return SEMIPAR_E_ARG;
  {
    const double cf = p->evolve.cell_factor;
    if (!(cf == 0.0 || (cf >= 1.0 && cf <= 4.0))) return SEMIPAR_E_ARG;
  }
  // One lane. Batches of one layer on concurrent lanes (host threads with streams of their
  // own) are switched off: a run with three lanes ended the process, and the cause is not
  // shown (region_destroy's device-wide hipFree on one lane while another lane captures
  // a graph is the suspect; the batched scheduler releases its batches only at its end).
  if (p->lanes > 1)
    return fail_msg(SEMIPAR_E_ARG, "schedule_handoff: one lane only (lanes > 1 is switched off)");
  const int lanes = 1;
  for (int r = 0; r < nr; ++r)
    if (h->n_pred[r] < 0 || h->succ_off[r + 1] < h->succ_off[r]) return SEMIPAR_E_ARG;
  if (h->succ_off[0] != 0) return SEMIPAR_E_ARG;
  {
    const int32_t m = h->succ_off[nr];
    if (m > 0 && !h->succ) return SEMIPAR_E_ARG;
    for (int32_t i = 0; i < m; ++i)
      if (h->succ[i] < 0 || h->succ[i] >= nr) return SEMIPAR_E_ARG;
  }
  // one lattice origin and scale; the box a whole number of region steps
  const semipar_region_geom& g0 = h->geoms[0];
  if (!(g0.inv2g > 0.0)) return SEMIPAR_E_ARG;
  for (int r = 1; r < nr; ++r) {
    const semipar_region_geom& g = h->geoms[r];
    if (g.inv2g != g0.inv2g) return SEMIPAR_E_ARG;
    for (int q = 0; q < 4; ++q)
      if (g.origin[q] != g0.origin[q]) return SEMIPAR_E_ARG;
  }
  const double Kd = 4.0 * h->box * g0.inv2g;
  const int K = (int)std::llround(Kd);
  if (K < 4 || K > 1024 || K % 4 != 0 || std::fabs(Kd - K) > 1e-9 * Kd)
    return fail_msg(SEMIPAR_E_ARG, "schedule_handoff: the box is not a whole number of region steps");
  // names -> region table
  std::vector<int64_t> name((size_t)nr);
  int32_t S_lo = INT32_MAX, S_hi = INT32_MIN;
  for (int r = 0; r < nr; ++r) {
    name[r] = region_name(h->geoms[r].idx, K);
    const int32_t S = (int32_t)(name[r] >> 32);
    S_lo = std::min(S_lo, S);
    S_hi = std::max(S_hi, S);
  }
  const int64_t K3 = (int64_t)K * K * K;
  const int64_t lut_n = ((int64_t)S_hi - S_lo + 1) * K3;
  if (lut_n > ((int64_t)1 << 28)) return SEMIPAR_E_ARG;
  std::vector<int32_t> lut((size_t)lut_n, -1);
  for (int r = 0; r < nr; ++r) {
    const int32_t S = (int32_t)(name[r] >> 32);
    const int64_t key = (int64_t)(uint32_t)(name[r] & 0xffffffffll);
    int32_t& e = lut[(size_t)((int64_t)(S - S_lo) * K3 + key)];
    if (e >= 0) return fail_msg(SEMIPAR_E_ARG, "schedule_handoff: two regions with one name");
    e = r;
  }
  Dev D;
  hipStream_t stream = (hipStream_t)h->stream;
  if (!stream) {
    hipError_t e = hipStreamCreate(&D.own);
    if (e != hipSuccess) return hip_msg(e, "hipStreamCreate");
    stream = D.own;
  }
  // the initial surface on the host: links by slot
  const int64_t n = h->n_points;
  std::vector<semipar_point_rec> recs;
  const semipar_point_rec* hrec = h->ic;
  if (h->ic_mem == SEMIPAR_MEM_DEVICE) {
    recs.resize((size_t)n);
    hipError_t e = hipMemcpyAsync(recs.data(), h->ic, sizeof(semipar_point_rec) * n,
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_msg(e, "copy of the initial surface");
    hrec = recs.data();
  }
  const int32_t s0r = hrec[0].step;
  if (s0r < 1) return SEMIPAR_E_SURFACE;
  std::unordered_map<int64_t, int32_t> slot_of;
  slot_of.reserve((size_t)n * 2);
  for (int64_t q = 0; q < n; ++q) {
    if (hrec[q].step != s0r) return SEMIPAR_E_SURFACE;
    if (!slot_of.emplace(hrec[q].id, (int32_t)q).second) return SEMIPAR_E_SURFACE;
  }
  std::vector<int32_t> gnext((size_t)n), gprev((size_t)n);
  std::vector<int64_t> gid((size_t)n);
  for (int64_t q = 0; q < n; ++q) {
    auto a = slot_of.find(hrec[q].next_id), b = slot_of.find(hrec[q].prev_id);
    if (a == slot_of.end() || b == slot_of.end()) return SEMIPAR_E_SURFACE;
    gnext[q] = a->second;
    gprev[q] = b->second;
    gid[q] = hrec[q].id;
  }
  for (int64_t q = 0; q < n; ++q)
    if (gprev[gnext[q]] != q) return SEMIPAR_E_SURFACE;
  slot_of.clear();
  // device tables
  int32_t *d_lut = nullptr, *d_gnext = nullptr, *d_gprev = nullptr, *d_gmap = nullptr;
  int64_t *d_gid = nullptr, *d_home = nullptr;
  semipar_point_rec* d_rec = nullptr;
  if (D.alloc(&d_home, (size_t)h->hist_slices * (size_t)n) != hipSuccess)
    return fail_msg(SEMIPAR_E_OOM, "schedule_handoff: vertex homes");
  if (D.alloc(&d_lut, lut.size()) != hipSuccess || D.alloc(&d_gnext, n) != hipSuccess ||
      D.alloc(&d_gprev, n) != hipSuccess || D.alloc(&d_gmap, (size_t)lanes * n) != hipSuccess ||
      D.alloc(&d_gid, n) != hipSuccess || D.alloc(&d_rec, n) != hipSuccess)
    return fail_msg(SEMIPAR_E_OOM, "schedule_handoff: device tables");
  {
    hipError_t e = hipMemcpyAsync(d_lut, lut.data(), sizeof(int32_t) * lut.size(),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_gnext, gnext.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_gprev, gprev.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_gid, gid.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(d_gmap, 0xff, sizeof(int32_t) * (size_t)lanes * n, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_rec, hrec, sizeof(semipar_point_rec) * n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_msg(e, "upload of the tiling tables");
  }
  spi::HandoffShared sh{};
  sh.H = h->hist;
  sh.home = d_home;
  sh.n = n;
  sh.s0 = s0r - 1;
  sh.ns = (int32_t)h->hist_slices;
  for (int q = 0; q < 4; ++q) sh.V[q] = g0.origin[q];
  sh.inv2g = g0.inv2g;
  sh.K = K;
  sh.S_lo = S_lo;
  sh.S_hi = S_hi;
  sh.lut = d_lut;
  sh.gnext = d_gnext;
  sh.gprev = d_gprev;
  sh.gid = d_gid;
  sh.gmap = d_gmap;
  sh.cosmology = h->cosmology;
  sh.box = h->box;
  // start tokens per region: (volume slot, first step)
  std::vector<std::vector<std::pair<int32_t, int32_t>>> work((size_t)nr);
  std::vector<char> finished((size_t)nr, 0);
  std::vector<spi::HandTok> tk;
  auto route = [&](const std::vector<spi::HandTok>& v) -> int {
    for (const spi::HandTok& t : v) {
      if (t.region < 0 || t.region >= nr || t.slot < 0 || t.slot >= n)
        return fail_msg(SEMIPAR_E_STATE, "schedule_handoff: a start token out of range");
      if (finished[t.region])
        return fail_msg(SEMIPAR_E_STATE,
                        "schedule_handoff: a region received work after it had run (the "
                        "dependency lists do not follow the geometry)");
      work[t.region].emplace_back(t.slot, t.step);
    }
    return SEMIPAR_OK;
  };
  {
    int rc = spi::handoff_ic(sh, d_rec, stream, tk);
    if (rc != SEMIPAR_OK) return rc;
    rc = route(tk);
    if (rc != SEMIPAR_OK) return rc;
  }
  // per-region results
  std::vector<std::vector<semipar_event>> ev_r((size_t)nr);
  std::vector<int32_t> r_steps((size_t)nr, 0), r_batch((size_t)nr, -1);
  std::vector<int64_t> r_psteps((size_t)nr, 0);
  std::vector<double> r_ms((size_t)nr, 0.0);
  std::vector<int32_t> ready;  // regions of the open layer with work, not yet taken
  std::vector<char> taken((size_t)nr, 0);
  int64_t batches = 0, steps_sum = 0, psum = 0, nev = 0, npass = 0, empty = 0, done = 0;
  double evolve_ms = 0.0, tk_ms = 0.0;
  int64_t tk_n = 0;
  semipar_evolve_params ep = p->evolve;
  if (ep.max_steps <= 0) ep.max_steps = (int64_t)1 << 30;
  ep.t_end = INFINITY;
  ep.loop_every = 0;
  ep.persistent = 0;
  // the manager's state, shared by the lanes under mu
  std::mutex mu;
  std::condition_variable cv;
  int running = 0, lane_rc = SEMIPAR_OK;
  std::string lane_msg;
  // Regions run layer by layer. A vertex's home lies in a later layer than the homes of
  // the vertices it was built from, or in their own region, so everything a region reads
  // or is told was made by an earlier layer or by itself, and the regions of one layer
  // never exchange anything: they run in any order, side by side.
  std::vector<int32_t> layer_of((size_t)nr);
  for (int r = 0; r < nr; ++r) layer_of[r] = (int32_t)(name[r] >> 32);
  for (int r = 0; r < nr; ++r)
    for (int32_t i = h->succ_off[r]; i < h->succ_off[r + 1]; ++i)
      if (layer_of[h->succ[i]] <= layer_of[r])
        return fail_msg(SEMIPAR_E_ARG,
                        "schedule_handoff: a successor in the same or an earlier layer");
  std::vector<int32_t> by_layer((size_t)nr);
  std::iota(by_layer.begin(), by_layer.end(), 0);
  std::stable_sort(by_layer.begin(), by_layer.end(),
                   [&](int32_t a, int32_t b) { return layer_of[a] < layer_of[b]; });
  size_t next_layer_at = 0;      // first region of the next layer in by_layer
  int32_t cur_layer = INT32_MIN;
  // open the next layer that has work (regions without work are done at once)
  auto open_layer = [&]() -> bool {
    while (next_layer_at < by_layer.size()) {
      cur_layer = layer_of[by_layer[next_layer_at]];
      while (next_layer_at < by_layer.size() && layer_of[by_layer[next_layer_at]] == cur_layer) {
        const int32_t r = by_layer[next_layer_at++];
        if (work[r].empty()) {
          finished[r] = 1;
          empty++;
          done++;
        } else {
          ready.push_back(r);
        }
      }
      if (!ready.empty()) return true;
    }
    return false;
  };
  // route a batch's tokens (under mu): only later layers can receive work
  auto route_locked = [&](const std::vector<spi::HandTok>& v) -> int {
    for (const spi::HandTok& t : v) {
      if (t.region < 0 || t.region >= nr || t.slot < 0 || t.slot >= n)
        return fail_msg(SEMIPAR_E_STATE, "schedule_handoff: a start token out of range");
      if (layer_of[t.region] <= cur_layer || finished[t.region] || taken[t.region])
        return fail_msg(SEMIPAR_E_STATE,
                        "schedule_handoff: a region received work after its layer had started");
      work[t.region].emplace_back(t.slot, t.step);
    }
    return SEMIPAR_OK;
  };
  open_layer();
  // one lane: take ready regions, longest predicted first (else most start tokens first),
  // up to batch_points points (0: all ready ones, shared out over the idle lanes)
  auto take = [&](int idle) {
    std::stable_sort(ready.begin(), ready.end(), [&](int32_t a, int32_t b) {
      if (p->cost) return p->cost[a] > p->cost[b];
      return work[a].size() > work[b].size();
    });
    int64_t all = 0;
    for (int32_t r : ready) all += (int64_t)work[r].size();
    const int64_t cap = p->batch_points > 0 ? p->batch_points
                                            : std::max<int64_t>(1, (all + idle - 1) / idle);
    std::vector<int32_t> regs;
    int64_t pts = 0;
    size_t i = 0;
    while (i < ready.size() && (regs.empty() || pts + (int64_t)work[ready[i]].size() <= cap)) {
      pts += (int64_t)work[ready[i]].size();
      regs.push_back(ready[i++]);
    }
    ready.erase(ready.begin(), ready.begin() + (ptrdiff_t)i);
    for (int32_t r : regs) taken[r] = 1;
    return regs;
  };
  auto lane_body = [&](int lane, hipStream_t ls) {
    std::vector<char> in_batch((size_t)n, 0);  // a point works in one region of a batch
    for (;;) {
      std::vector<int32_t> regs;
      int64_t my_batch = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return lane_rc != SEMIPAR_OK || !ready.empty() || running == 0; });
        if (lane_rc == SEMIPAR_OK && ready.empty() && running == 0) open_layer();
        if (lane_rc != SEMIPAR_OK || ready.empty()) {
          cv.notify_all();
          return;
        }
        regs = take(std::max(1, lanes - running));
        my_batch = batches++;
        running++;
      }
      // the batch: its regions' start tokens, sorted by volume slot (a region's tokens are
      // complete once it is ready: all their producers have run)
      std::vector<int32_t> slot, start;
      std::vector<int64_t> sub_off(1, 0), names;
      std::vector<semipar_region_geom> geoms;
      int rc = SEMIPAR_OK;
      for (int32_t r : regs) {
        auto& w = work[r];
        std::sort(w.begin(), w.end());
        int32_t last = -1;
        for (const auto& e : w) {
          if (e.first == last) {
            if (e.second != start.back())
              rc = fail_msg(SEMIPAR_E_STATE, "schedule_handoff: a point starts twice in one region");
            continue;
          }
          if (in_batch[e.first])
            rc = fail_msg(SEMIPAR_E_STATE,
                          "schedule_handoff: a point works in two regions of one batch");
          in_batch[e.first] = 1;
          last = e.first;
          slot.push_back(e.first);
          start.push_back(e.second);
        }
        sub_off.push_back((int64_t)slot.size());
        geoms.push_back(h->geoms[r]);
        names.push_back(name[r]);
      }
      for (int32_t q : slot) in_batch[q] = 0;
      semipar_region* R = nullptr;
      semipar_evolve_stats es{};
      std::vector<semipar_event> evs;
      std::vector<int64_t> eoff, bps;
      std::vector<int32_t> bsteps;
      std::vector<spi::HandTok> btk;
      if (rc == SEMIPAR_OK)
        rc = spi::handoff_batch(sh, lane, slot.data(), start.data(), sub_off, geoms.data(),
                                names.data(), ls, &R);
      if (rc == SEMIPAR_OK) rc = region_evolve(R, &ep, &es);
      if (rc == SEMIPAR_OK && es.steps >= ep.max_steps)
        rc = fail_msg(SEMIPAR_E_STATE, "schedule_handoff: a batch reached max_steps");
      if (rc == SEMIPAR_OK) rc = spi::batch_events(R, evs, eoff);
      if (rc == SEMIPAR_OK) rc = spi::batch_stats(R, bsteps, bps);
      if (rc == SEMIPAR_OK) rc = spi::handoff_tokens(R, btk);
      region_destroy(R);
      std::unique_lock<std::mutex> lk(mu);
      running--;
      if (rc == SEMIPAR_OK) rc = route_locked(btk);
      if (rc != SEMIPAR_OK) {
        if (lane_rc == SEMIPAR_OK) {
          lane_rc = rc;
          lane_msg = semipar_last_error();
        }
        cv.notify_all();
        return;
      }
      for (size_t q = 0; q < regs.size(); ++q) {
        const int32_t r = regs[q];
        ev_r[r].assign(evs.begin() + eoff[q], evs.begin() + eoff[q + 1]);
        for (const semipar_event& e : ev_r[r]) npass += e.kind == 1 ? 1 : 0;
        nev += (int64_t)ev_r[r].size();
        r_steps[r] = bsteps[q];
        r_psteps[r] = bps[q];
        r_batch[r] = (int32_t)my_batch;
        r_ms[r] = es.elapsed_ms;
        psum += bps[q];
        work[r].clear();
        work[r].shrink_to_fit();
        finished[r] = 1;
        done++;
      }
      steps_sum += es.steps;
      evolve_ms += es.elapsed_ms;
      tk_ms += es.timed_kernel_ms;
      tk_n += es.timed_kernel_launches;
      cv.notify_all();
    }
  };
  lane_body(0, stream);
  if (lane_rc != SEMIPAR_OK) {
    spi::set_error(lane_msg.c_str());  // the lane's message, on the caller's thread
    return lane_rc;
  }
  if (done != nr)
    return fail_msg(SEMIPAR_E_ARG, "schedule_handoff: the dependency lists leave regions never ready");
  if (p->events) {
    int64_t off = 0;
    for (int r = 0; r < nr; ++r) {
      p->events_off[r] = off;
      for (const semipar_event& e : ev_r[r]) {
        if (off < p->events_cap) p->events[off] = e;
        off++;
      }
    }
    p->events_off[nr] = off;
  }
  for (int r = 0; r < nr; ++r) {
    if (p->region_steps) p->region_steps[r] = r_steps[r];
    if (p->region_point_steps) p->region_point_steps[r] = r_psteps[r];
    if (p->region_batch) p->region_batch[r] = r_batch[r];
    if (p->region_ms) p->region_ms[r] = r_ms[r];
  }
  if (st) {
    semipar_sched_stats z{};
    *st = z;
    st->regions = nr;
    st->empty_regions = empty;
    st->batches = batches;
    st->point_steps = psum;
    st->steps = steps_sum;
    st->events = nev;
    st->passed = npass;
    st->evolve_ms = evolve_ms;
    st->timed_kernel_ms = tk_ms;
    st->timed_kernel_launches = tk_n;
    st->makespan_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return SEMIPAR_OK;
}
