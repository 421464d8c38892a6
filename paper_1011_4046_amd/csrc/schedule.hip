// schedule.hip -- many regions on one GPU: ready queue, empty fast path, launch batches.
//
// Paper, Section "Implementation": a manager keeps the set of regions whose
// predecessors have all finished and hands them to idle workers; a region whose
// initial surfaces hold no string is only noted. Section "Performance": the elapsed
// time is set by the most difficult regions, which is why uneven regions are packed
// by predicted cost here.
//
// On one GPU the "workers" are launch batches: every ready region of a wave goes into
// a batch region (one set of kernels over the points of all its sub-regions), and a
// batch runs until all its sub-regions have stopped. Regions are ordered by predicted
// lattice steps (cost model) or, without a prediction, by point count, and cut into
// batches of at most batch_points points, so that regions finishing after similar
// numbers of steps share a launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "internal.h"
#include "semipar.h"

#define RCCHK_R(x)            \
  do {                        \
    int rc_ = (x);            \
    if (rc_ != 0) return rc_; \
  } while (0)

namespace {

struct Slab {
  int64_t base = 0;  // first output record of the region
};

int check_tiling(const semipar_tiling* t) {
  if (!t || t->n_regions < 0 || !(t->box > 0.0) || t->cosmology < 0 || t->cosmology > 2)
    return SEMIPAR_E_ARG;
  if (t->n_regions > 0 && (!t->surfaces || !t->geoms)) return SEMIPAR_E_ARG;
  for (int r = 0; r < t->n_regions; ++r) {
    const semipar_surface& s = t->surfaces[r];
    if (s.n < 0 || (s.n > 0 && !s.recs)) return SEMIPAR_E_ARG;
    if (s.mem != SEMIPAR_MEM_HOST && s.mem != SEMIPAR_MEM_DEVICE) return SEMIPAR_E_ARG;
    if (!(t->geoms[r].inv2g > 0.0)) return SEMIPAR_E_ARG;
  }
  if (t->n_pred) {
    if (!t->succ_off) return SEMIPAR_E_ARG;
    for (int r = 0; r < t->n_regions; ++r)
      if (t->n_pred[r] < 0 || t->succ_off[r + 1] < t->succ_off[r]) return SEMIPAR_E_ARG;
    const int32_t m = t->succ_off[t->n_regions];
    if (m > 0 && !t->succ) return SEMIPAR_E_ARG;
    for (int32_t i = 0; i < m; ++i)
      if (t->succ[i] < 0 || t->succ[i] >= t->n_regions) return SEMIPAR_E_ARG;
  }
  return SEMIPAR_OK;
}

semipar_region_desc batch_desc(const semipar_tiling* t, const std::vector<int32_t>& regs,
                               std::vector<semipar_region_geom>& g) {
  g.resize(regs.size());
  for (size_t i = 0; i < regs.size(); ++i) g[i] = t->geoms[regs[i]];
  semipar_region_desc d{};
  d.cosmology = t->cosmology;
  d.bounded = 1;
  d.box = t->box;
  d.stream = t->stream;
  d.n_sub = (int32_t)regs.size();
  d.sub = g.data();
  return d;
}

struct Runner {
  const semipar_tiling* t;
  const semipar_sched_params* p;
  std::vector<Slab> slab;
  std::vector<std::vector<semipar_event>> ev;  // per region
  std::vector<std::vector<semipar_loop>> lp;   // per region
  semipar_sched_stats acc{};
  int32_t batch_id = 0;
  semipar_point_rec* tmp = nullptr;
  int64_t tmp_cap = 0;

  ~Runner() {
    if (tmp) (void)hipFree(tmp);
  }

  void log_region(int32_t r, int32_t steps, int64_t psteps, int32_t batch, double ms) {
    if (p->region_steps) p->region_steps[r] = steps;
    if (p->region_point_steps) p->region_point_steps[r] = psteps;
    if (p->region_batch) p->region_batch[r] = batch;
    if (p->region_ms) p->region_ms[r] = ms;
  }

  // plain policy: one region per launch sequence, its own region object
  int run_plain(int32_t r) {
    const semipar_surface& s = t->surfaces[r];
    semipar_region_desc d{};
    d.cosmology = t->cosmology;
    d.bounded = 1;
    d.box = t->box;
    d.stream = t->stream;
    for (int i = 0; i < 4; ++i) {
      d.idx[i] = t->geoms[r].idx[i];
      d.origin[i] = t->geoms[r].origin[i];
    }
    d.inv2g = t->geoms[r].inv2g;
    semipar_region* reg = nullptr;
    int rc = region_init_from_surfaces(&d, &s, 1, &reg);
    if (rc != SEMIPAR_OK) return rc;
    semipar_evolve_stats es{};
    rc = region_evolve(reg, &p->evolve, &es);
    int64_t n[4] = {0, 0, 0, 0};
    if (rc == SEMIPAR_OK && p->out) {
      rc = region_emit_final_surfaces(reg, nullptr, nullptr, n, p->out_mem);
      if (rc == SEMIPAR_OK) {
        semipar_point_rec* o[4];
        int64_t off = slab[r].base;
        for (int f = 0; f < 4; ++f) {
          o[f] = p->out + off;
          if (p->out_off) p->out_off[4 * r + f] = off;
          off += n[f];
        }
        rc = region_emit_final_surfaces(reg, o, n, n, p->out_mem);
      }
    }
    if (rc == SEMIPAR_OK && p->events) {
      int64_t ne = 0;
      rc = region_events(reg, nullptr, 0, &ne);
      if (rc == SEMIPAR_OK) {
        ev[r].resize((size_t)ne);
        if (ne > 0) rc = region_events(reg, ev[r].data(), ne, &ne);
      }
    }
    if (rc == SEMIPAR_OK && p->loops) {
      int64_t nl = 0;
      rc = region_loops(reg, nullptr, 0, &nl);
      if (rc == SEMIPAR_OK) {
        lp[r].resize((size_t)nl);
        if (nl > 0) rc = region_loops(reg, lp[r].data(), nl, &nl);
      }
    }
    std::vector<int32_t> steps;
    std::vector<int64_t> ps;
    if (rc == SEMIPAR_OK) rc = spi::batch_stats(reg, steps, ps);
    region_destroy(reg);
    if (rc != SEMIPAR_OK) return rc;
    acc.point_steps += es.point_steps;
    acc.steps += es.steps;
    acc.evolve_ms += es.elapsed_ms;
    acc.timed_kernel_ms += es.timed_kernel_ms;
    acc.timed_kernel_launches += es.timed_kernel_launches;
    acc.loops += es.loops;
    acc.passed += es.passed;
    acc.batches += 1;
    log_region(r, steps[0], ps[0], batch_id++, es.elapsed_ms);
    return SEMIPAR_OK;
  }

  // batched policy: regs share one batch region. A batch goes through three phases:
  // build (init from the surfaces, step buffers and log sized up front), evolve, and
  // finish (per-region records, events and logs; destroy).
  struct Batch {
    std::vector<int32_t> regs;
    std::vector<int64_t> n;
    semipar_region* reg = nullptr;
    semipar_evolve_stats es{};
    int rc = SEMIPAR_OK;
    double cost = 0.0;  // predicted device time, for assigning batches to lanes
  };

  int build_batch(Batch& b, void* stream) {
    std::vector<semipar_region_geom> g;
    semipar_region_desc d = batch_desc(t, b.regs, g);
    d.stream = stream;
    std::vector<semipar_surface> in(b.regs.size());
    b.n.resize(b.regs.size());
    for (size_t i = 0; i < b.regs.size(); ++i) {
      in[i] = t->surfaces[b.regs[i]];
      b.n[i] = in[i].n;
    }
    int rc = region_init_from_surfaces(&d, in.data(), (int)in.size(), &b.reg);
    if (rc == SEMIPAR_OK) rc = spi::region_prepare(b.reg, &p->evolve);
    return rc;
  }

  int finish_batch(Batch& b) {
    int rc = b.rc;
    semipar_region* reg = b.reg;
    const auto& regs = b.regs;
    int64_t total = 0;
    for (int64_t x : b.n) total += x;
    if (rc == SEMIPAR_OK && p->out && total > 0) {
      if (tmp_cap < total) {
        if (tmp) (void)hipFree(tmp);
        tmp = nullptr;
        tmp_cap = 0;
        if (hipMalloc(&tmp, sizeof(semipar_point_rec) * total) != hipSuccess) rc = SEMIPAR_E_OOM;
        else tmp_cap = total;
      }
      std::vector<int64_t> cnt;
      if (rc == SEMIPAR_OK) rc = spi::batch_emit(reg, tmp, cnt);
      const hipMemcpyKind kind =
          p->out_mem == SEMIPAR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
      hipStream_t s = spi::region_stream(reg);
      int64_t src = 0;
      for (size_t i = 0; i < regs.size() && rc == SEMIPAR_OK; ++i) {
        const int32_t r = regs[i];
        const int64_t nr = b.n[i];
        int64_t off = slab[r].base;
        for (int f = 0; f < 4; ++f) {
          if (p->out_off) p->out_off[4 * r + f] = off;
          off += cnt[4 * i + f];
        }
        if (nr > 0 && hipMemcpyAsync(p->out + slab[r].base, tmp + src,
                                     sizeof(semipar_point_rec) * nr, kind, s) != hipSuccess)
          rc = SEMIPAR_E_HIP;
        src += nr;
      }
      if (rc == SEMIPAR_OK && hipStreamSynchronize(s) != hipSuccess) rc = SEMIPAR_E_HIP;
    }
    if (rc == SEMIPAR_OK && p->events) {
      std::vector<semipar_event> e;
      std::vector<int64_t> off;
      rc = spi::batch_events(reg, e, off);
      for (size_t i = 0; i < regs.size() && rc == SEMIPAR_OK; ++i)
        ev[regs[i]].assign(e.begin() + off[i], e.begin() + off[i + 1]);
    }
    if (rc == SEMIPAR_OK && p->loops) {
      std::vector<semipar_loop> l;
      std::vector<int64_t> off;
      rc = spi::batch_loops(reg, l, off);
      for (size_t i = 0; i < regs.size() && rc == SEMIPAR_OK; ++i)
        lp[regs[i]].assign(l.begin() + off[i], l.begin() + off[i + 1]);
    }
    std::vector<int32_t> steps;
    std::vector<int64_t> ps;
    if (rc == SEMIPAR_OK) rc = spi::batch_stats(reg, steps, ps);
    region_destroy(reg);
    b.reg = nullptr;
    if (rc != SEMIPAR_OK) return rc;
    const semipar_evolve_stats& es = b.es;
    acc.point_steps += es.point_steps;
    acc.steps += es.steps;
    acc.evolve_ms += es.elapsed_ms;
    acc.timed_kernel_ms += es.timed_kernel_ms;
    acc.timed_kernel_launches += es.timed_kernel_launches;
    acc.loops += es.loops;
    acc.passed += es.passed;
    acc.batches += 1;
    for (size_t i = 0; i < regs.size(); ++i)
      log_region(regs[i], steps[i], ps[i], batch_id, es.elapsed_ms);
    batch_id++;
    return SEMIPAR_OK;
  }

  // Run the batches of one wave: with one lane, one after another on the tiling's
  // stream; with L lanes, all batches are built first (nothing is freed while kernels
  // run, since hipFree waits for the whole device), then L host threads each evolve
  // their batches on a stream of their own, longest predicted batch first onto the
  // least loaded lane, and the results are collected afterwards.
  int run_batches(std::vector<Batch>& bs) {
    const int lanes = std::max(1, std::min<int>(p->lanes, (int)bs.size()));
    if (lanes == 1) {
      for (Batch& b : bs) {
        int rc = build_batch(b, t->stream);
        if (rc == SEMIPAR_OK) rc = region_evolve(b.reg, &p->evolve, &b.es);
        b.rc = rc;
        RCCHK_R(finish_batch(b));
      }
      return SEMIPAR_OK;
    }
    std::vector<hipStream_t> ls(lanes, nullptr);
    hipEvent_t ready = nullptr;
    int rc = SEMIPAR_OK;
    for (int l = 0; l < lanes && rc == SEMIPAR_OK; ++l)
      if (hipStreamCreateWithFlags(&ls[l], hipStreamNonBlocking) != hipSuccess) rc = SEMIPAR_E_HIP;
    if (rc == SEMIPAR_OK && t->stream) {
      // device-resident surfaces may still be in flight on the caller's stream
      if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
          hipEventRecord(ready, (hipStream_t)t->stream) != hipSuccess)
        rc = SEMIPAR_E_HIP;
      for (int l = 0; l < lanes && rc == SEMIPAR_OK; ++l)
        if (hipStreamWaitEvent(ls[l], ready, 0) != hipSuccess) rc = SEMIPAR_E_HIP;
    }
    // longest processing time first onto the least loaded lane
    std::vector<int> order(bs.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return bs[a].cost > bs[b].cost; });
    std::vector<std::vector<int>> work(lanes);
    std::vector<double> load(lanes, 0.0);
    for (int i : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      work[l].push_back(i);
      load[l] += bs[i].cost;
    }
    for (int l = 0; l < lanes && rc == SEMIPAR_OK; ++l)
      for (int i : work[l]) {
        rc = build_batch(bs[i], ls[l]);
        if (rc != SEMIPAR_OK) break;
      }
    if (rc == SEMIPAR_OK) {
      std::vector<std::thread> th;
      for (int l = 0; l < lanes; ++l)
        th.emplace_back([&, l]() {
          for (int i : work[l]) {
            bs[i].rc = region_evolve(bs[i].reg, &p->evolve, &bs[i].es);
            if (bs[i].rc != SEMIPAR_OK) break;
          }
        });
      for (auto& x : th) x.join();
      for (int l = 0; l < lanes && rc == SEMIPAR_OK; ++l)
        for (int i : work[l])
          if (bs[i].rc != SEMIPAR_OK) rc = bs[i].rc;
    }
    for (int l = 0; l < lanes && rc == SEMIPAR_OK; ++l)
      for (int i : work[l]) {
        rc = finish_batch(bs[i]);
        if (rc != SEMIPAR_OK) break;
      }
    for (Batch& b : bs)
      if (b.reg) {
        region_destroy(b.reg);
        b.reg = nullptr;
      }
    for (hipStream_t x : ls)
      if (x) (void)hipStreamDestroy(x);
    if (ready) (void)hipEventDestroy(ready);
    return rc;
  }

  // one wave of ready regions
  int run_wave(std::vector<int32_t> ready) {
    std::vector<int32_t> live;
    for (int32_t r : ready) {
      if (t->surfaces[r].n == 0) {
        // empty fast path: nothing to simulate, nothing to emit
        acc.empty_regions += 1;
        if (p->out_off)
          for (int f = 0; f < 4; ++f) p->out_off[4 * r + f] = slab[r].base;
        log_region(r, 0, 0, -1, 0.0);
      } else {
        live.push_back(r);
      }
      acc.regions += 1;
    }
    if (p->policy == SEMIPAR_SCHED_PLAIN) {
      for (int32_t r : live) RCCHK_R(run_plain(r));
      return SEMIPAR_OK;
    }
    // batched: longest predicted first (steps from the cost model, else points)
    std::stable_sort(live.begin(), live.end(), [&](int32_t a, int32_t b) {
      if (p->cost) return p->cost[a] > p->cost[b];
      return t->surfaces[a].n > t->surfaces[b].n;
    });
    std::vector<Batch> bs;
    if (p->pack == SEMIPAR_PACK_WORK && p->cost && !live.empty()) {
      // equal shares of the predicted point-steps, in decreasing cost order
      double work = 0.0;
      int64_t total = 0;
      for (int32_t r : live) {
        work += (double)t->surfaces[r].n * std::max(1.0, (double)p->cost[r]);
        total += t->surfaces[r].n;
      }
      int64_t nb = std::max<int64_t>(1, p->lanes);
      if (p->batch_points > 0) nb = std::max(nb, (total + p->batch_points - 1) / p->batch_points);
      nb = std::min<int64_t>(nb, (int64_t)live.size());
      const double share = work / (double)nb;
      double done = 0.0;
      for (int32_t r : live) {
        if (bs.empty() || ((int64_t)bs.size() < nb && done >= share * (double)bs.size()))
          bs.emplace_back();
        bs.back().regs.push_back(r);
        done += (double)t->surfaces[r].n * std::max(1.0, (double)p->cost[r]);
      }
    } else {
      int64_t pts = 0;
      for (int32_t r : live) {
        const int64_t nr = t->surfaces[r].n;
        if (bs.empty() || (p->batch_points > 0 && pts + nr > p->batch_points)) {
          bs.emplace_back();
          pts = 0;
        }
        bs.back().regs.push_back(r);
        pts += nr;
      }
    }
    // predicted device time of a batch: its points, for as many steps as its longest
    // region needs (steps from the cost model; without one, the points alone)
    for (Batch& b : bs) {
      double np = 0.0, mx = 1.0;
      for (int32_t r : b.regs) {
        np += (double)t->surfaces[r].n;
        if (p->cost) mx = std::max(mx, (double)p->cost[r]);
      }
      b.cost = np * mx;
    }
    return run_batches(bs);
  }
};

}  // namespace

extern "C" {

int schedule_regions(const semipar_tiling* t, const semipar_sched_params* p,
                     semipar_sched_stats* st) {
  if (!p) return SEMIPAR_E_ARG;
  int rc = check_tiling(t);
  if (rc != SEMIPAR_OK) return rc;
  if (p->policy != SEMIPAR_SCHED_PLAIN && p->policy != SEMIPAR_SCHED_BATCHED) return SEMIPAR_E_ARG;
  if (p->lanes < 0 || p->lanes > 16) return SEMIPAR_E_ARG;
  if (p->pack != SEMIPAR_PACK_POINTS && p->pack != SEMIPAR_PACK_WORK) return SEMIPAR_E_ARG;
  if (p->batch_points < 0 || (p->out && p->out_mem != SEMIPAR_MEM_HOST &&
                              p->out_mem != SEMIPAR_MEM_DEVICE))
    return SEMIPAR_E_ARG;
  if (p->events && (!p->events_off || p->events_cap < 0)) return SEMIPAR_E_ARG;
  if (p->loops && (!p->loops_off || p->loops_cap < 0)) return SEMIPAR_E_ARG;
  if (p->evolve.loop_every < 0) return SEMIPAR_E_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  Runner R;
  R.t = t;
  R.p = p;
  const int nr = t->n_regions;
  R.slab.resize(nr);
  R.ev.resize(nr);
  R.lp.resize(nr);
  int64_t base = 0;
  for (int r = 0; r < nr; ++r) {
    R.slab[r].base = base;
    base += t->surfaces[r].n;
  }
  if (p->out_off) p->out_off[4 * (int64_t)nr] = base;
  // ready queue: regions whose predecessors have all finished, wave by wave
  std::vector<int32_t> pending(nr, 0);
  std::vector<int32_t> ready;
  for (int r = 0; r < nr; ++r) {
    pending[r] = t->n_pred ? t->n_pred[r] : 0;
    if (pending[r] == 0) ready.push_back(r);
  }
  int done = 0;
  while (!ready.empty()) {
    rc = R.run_wave(ready);
    if (rc != SEMIPAR_OK) return rc;
    done += (int)ready.size();
    std::vector<int32_t> next;
    if (t->n_pred)
      for (int32_t r : ready)
        for (int32_t i = t->succ_off[r]; i < t->succ_off[r + 1]; ++i)
          if (--pending[t->succ[i]] == 0) next.push_back(t->succ[i]);
    std::sort(next.begin(), next.end());
    ready.swap(next);
  }
  if (done != nr) {
    spi::set_error("schedule_regions: the predecessor counts leave regions that never become ready");
    return SEMIPAR_E_ARG;
  }
  // event lists, region by region
  int64_t ne = 0;
  for (int r = 0; r < nr; ++r) {
    const int64_t m = (int64_t)R.ev[r].size();
    if (p->events) {
      p->events_off[r] = ne;
      const int64_t fit = std::max<int64_t>(0, std::min(m, p->events_cap - ne));
      if (fit > 0) memcpy(p->events + ne, R.ev[r].data(), sizeof(semipar_event) * fit);
    }
    ne += m;
  }
  if (p->events) p->events_off[nr] = ne;
  R.acc.events = ne;
  int64_t nl = 0;
  for (int r = 0; r < nr; ++r) {
    const int64_t m = (int64_t)R.lp[r].size();
    if (p->loops) {
      p->loops_off[r] = nl;
      const int64_t fit = std::max<int64_t>(0, std::min(m, p->loops_cap - nl));
      if (fit > 0) memcpy(p->loops + nl, R.lp[r].data(), sizeof(semipar_loop) * fit);
    }
    nl += m;
  }
  if (p->loops) p->loops_off[nr] = nl;
  R.acc.makespan_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = R.acc;
  return SEMIPAR_OK;
}

int semipar_region_features(const semipar_tiling* t, float* feat) {
  int rc = check_tiling(t);
  if (rc != SEMIPAR_OK || !feat) return SEMIPAR_E_ARG;
  if (t->n_regions == 0) return SEMIPAR_OK;
  // surfaces in device memory: read in place; otherwise through a batch of all regions
  bool on_device = true;
  for (int r = 0; r < t->n_regions; ++r)
    on_device = on_device && (t->surfaces[r].n == 0 || t->surfaces[r].mem == SEMIPAR_MEM_DEVICE);
  if (on_device) return spi::surface_features(t, feat);
  std::vector<int32_t> all((size_t)t->n_regions);
  std::iota(all.begin(), all.end(), 0);
  std::vector<semipar_region_geom> g;
  semipar_region_desc d = batch_desc(t, all, g);
  semipar_region* reg = nullptr;
  rc = region_init_from_surfaces(&d, t->surfaces, t->n_regions, &reg);
  if (rc != SEMIPAR_OK) return rc;
  rc = spi::batch_features(reg, feat);
  region_destroy(reg);
  return rc;
}

}  // extern "C"
