// schedule.hip -- many regions on one GPU: ready queue, empty fast path, launch batches.
//
// Paper, Section "Implementation": a manager keeps the set of regions whose
// predecessors have all finished and hands them to idle workers; a region whose
// initial surfaces hold no string is only noted. Section "Performance": the elapsed
// time is set by the most difficult regions, which is why uneven regions are packed
// by predicted cost here.
//
// On one GPU the "workers" are launch batches: ready regions go into a batch region
// (one set of kernels over the points of all its sub-regions), and a batch runs until
// all its sub-regions have stopped. Regions are ordered by predicted lattice steps (cost
// model) or, without a prediction, by point count, and cut into batches of at most
// batch_points points, so that regions finishing after similar numbers of steps share a
// launch. The manager's bookkeeping -- predecessor counts, successor lists, the ring of
// ready regions and the empty-region fast path -- is on the device (k_dag_release); a
// finished batch releases its regions' successors at once, so a region starts as soon
// as its own predecessors are done.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
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

// A failed HIP call: its text for semipar_last_error, and SEMIPAR_E_HIP.
int hip_err(hipError_t e, const char* what) {
  char msg[200];
  snprintf(msg, sizeof(msg), "schedule_regions: %s failed: %s", what, hipGetErrorString(e));
  spi::set_error(msg);
  return SEMIPAR_E_HIP;
}

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

// ---------------------------------------------------------------------------------
// the ready queue on the device
// ---------------------------------------------------------------------------------
// Per region: predecessors still running (pending), successors (CSR), and whether its
// initial surface holds no string. A region enters the ready ring exactly once, when
// its count reaches zero; a ready region without string completes at once (the paper's
// empty regions are only noted) and so releases its own successors in the same kernel.
constexpr int DAG_NT = 1024;

// Release the successors of the `nfin` regions in fin (seed = 1: instead, make every
// region with no pending predecessor ready). Regions that become ready are appended to
// ring (tail at ctr[0]); ready regions without string are followed through at once,
// breadth first, on the worklist `work` (nr entries). One workgroup.
__global__ __launch_bounds__(DAG_NT) void k_dag_release(
    const int32_t* __restrict__ fin, int nfin, int seed, int nr, int32_t* __restrict__ pending,
    const int32_t* __restrict__ succ_off, const int32_t* __restrict__ succ,
    const uint8_t* __restrict__ empty, int32_t* __restrict__ ring, int32_t* __restrict__ ctr,
    int32_t* __restrict__ work) {
  __shared__ int s_n;
  const int t = threadIdx.x;
  if (t == 0) s_n = 0;
  __syncthreads();
  auto ready = [&](int32_t r) {
    ring[atomicAdd(&ctr[0], 1)] = r;
    if (empty[r]) work[atomicAdd(&s_n, 1)] = r;
  };
  auto release = [&](int32_t r) {
    for (int32_t e = succ_off[r]; e < succ_off[r + 1]; ++e)
      if (atomicSub(&pending[succ[e]], 1) == 1) ready(succ[e]);
  };
  if (seed) {
    for (int r = t; r < nr; r += DAG_NT)
      if (pending[r] == 0) ready(r);
  } else {
    for (int i = t; i < nfin; i += DAG_NT) release(fin[i]);
  }
  int head = 0;
  for (;;) {
    __syncthreads();
    const int end = s_n;
    __syncthreads();  // every thread has read the end before new regions are appended
    if (head >= end) break;
    for (int i = head + t; i < end; i += DAG_NT) release(work[i]);
    head = end;
  }
}

struct DagDev {
  int32_t *pending = nullptr, *succ_off = nullptr, *succ = nullptr, *ring = nullptr;
  int32_t *ctr = nullptr, *work = nullptr, *fin = nullptr;
  uint8_t* empty = nullptr;
  ~DagDev() {
    for (void* q : {(void*)pending, (void*)succ_off, (void*)succ, (void*)ring, (void*)ctr,
                    (void*)work, (void*)fin, (void*)empty})
      if (q) (void)hipFree(q);
  }
};

// A region's share of a list that a whole batch brought back from the device: the
// batch's list stays as it came and each of its regions keeps where its part lies, so
// that the entries are copied once, into the caller's list, when the schedule ends.
template <class T>
struct Part {
  std::shared_ptr<const std::vector<T>> buf;
  int64_t off = 0, n = 0;
  const T* data() const { return buf ? buf->data() + off : nullptr; }
  int64_t size() const { return n; }
};

template <class T>
void share_out(std::vector<T>&& list, const std::vector<int64_t>& off,
               const std::vector<int32_t>& regs, std::vector<Part<T>>& parts) {
  auto buf = std::make_shared<const std::vector<T>>(std::move(list));
  for (size_t i = 0; i < regs.size(); ++i) parts[regs[i]] = Part<T>{buf, off[i], off[i + 1] - off[i]};
}

struct Runner {
  const semipar_tiling* t;
  const semipar_sched_params* p;
  std::vector<Slab> slab;
  std::vector<Part<semipar_event>> ev;  // per region
  std::vector<Part<semipar_loop>> lp;   // per region
  semipar_sched_stats acc{};
  int32_t batch_id = 0;

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
        std::vector<semipar_event> e((size_t)ne);
        if (ne > 0) rc = region_events(reg, e.data(), ne, &ne);
        if (rc == SEMIPAR_OK) share_out(std::move(e), {0, ne}, {r}, ev);
      }
    }
    if (rc == SEMIPAR_OK && p->loops) {
      int64_t nl = 0;
      rc = region_loops(reg, nullptr, 0, &nl);
      if (rc == SEMIPAR_OK) {
        std::vector<semipar_loop> l((size_t)nl);
        if (nl > 0) rc = region_loops(reg, l.data(), nl, &nl);
        if (rc == SEMIPAR_OK) share_out(std::move(l), {0, nl}, {r}, lp);
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
    std::string msg;    // the lane's error message when rc is not SEMIPAR_OK
    double cost = 0.0;  // predicted device time, for assigning batches to lanes
    std::vector<int32_t> steps;  // per region: slices advanced (after harvest)
    std::vector<int64_t> ps;     // per region: point-steps (after harvest)
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

  // Results of an evolved batch, taken on its lane as soon as it has evolved, so that
  // they overlap the other lanes' steps: records into the output (device output: written
  // in place; host output: through the lane's device staging buffer), events and loop
  // logs into the per-region lists, per-region step counts. Every device temporary is
  // stream-ordered on the batch's stream, so nothing here waits for another lane.
  int harvest(Batch& b, semipar_point_rec*& stage, int64_t& stage_cap) {
    semipar_region* reg = b.reg;
    const auto& regs = b.regs;
    int64_t total = 0;
    for (int64_t x : b.n) total += x;
    int rc = SEMIPAR_OK;
    if (p->out && total > 0) {
      std::vector<int64_t> cnt;
      if (p->out_mem == SEMIPAR_MEM_DEVICE) {
        std::vector<int64_t> base(regs.size());
        for (size_t i = 0; i < regs.size(); ++i) base[i] = slab[regs[i]].base;
        rc = spi::batch_emit(reg, p->out, cnt, base.data());
      } else {
        if (stage_cap < total) {
          if (stage) (void)hipFree(stage);
          stage = nullptr;
          stage_cap = 0;
          if (hipMalloc(&stage, sizeof(semipar_point_rec) * total) != hipSuccess) {
            spi::set_error("schedule_regions: device allocation of the output staging failed");
            return SEMIPAR_E_OOM;
          }
          stage_cap = total;
        }
        rc = spi::batch_emit(reg, stage, cnt);
        hipStream_t s = spi::region_stream(reg);
        int64_t src = 0;
        for (size_t i = 0; i < regs.size() && rc == SEMIPAR_OK; ++i) {
          const int64_t nr = b.n[i];
          if (nr > 0) {
            const hipError_t e =
                hipMemcpyAsync(p->out + slab[regs[i]].base, stage + src,
                               sizeof(semipar_point_rec) * nr, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) rc = hip_err(e, "record copy to the host");
          }
          src += nr;
        }
        if (rc == SEMIPAR_OK) {
          const hipError_t e = hipStreamSynchronize(s);
          if (e != hipSuccess) rc = hip_err(e, "record copy to the host");
        }
      }
      for (size_t i = 0; i < regs.size() && rc == SEMIPAR_OK; ++i) {
        const int32_t r = regs[i];
        int64_t off = slab[r].base;
        for (int f = 0; f < 4; ++f) {
          if (p->out_off) p->out_off[4 * r + f] = off;
          off += cnt[4 * i + f];
        }
      }
    }
    if (rc == SEMIPAR_OK && p->events) {
      std::vector<semipar_event> e;
      std::vector<int64_t> off;
      rc = spi::batch_events(reg, e, off);
      if (rc == SEMIPAR_OK) share_out(std::move(e), off, regs, ev);
    }
    if (rc == SEMIPAR_OK && p->loops) {
      std::vector<semipar_loop> l;
      std::vector<int64_t> off;
      rc = spi::batch_loops(reg, l, off);
      if (rc == SEMIPAR_OK) share_out(std::move(l), off, regs, lp);
    }
    if (rc == SEMIPAR_OK) rc = spi::batch_stats(reg, b.steps, b.ps);
    return rc;
  }

  // A harvested batch: totals, per-region log, and the batch region released (releasing
  // device memory waits for the whole device, so this runs once all batches are done).
  int finish_batch(Batch& b) {
    if (b.reg) region_destroy(b.reg);
    b.reg = nullptr;
    if (b.rc != SEMIPAR_OK) return b.rc;
    const semipar_evolve_stats& es = b.es;
    acc.point_steps += es.point_steps;
    acc.steps += es.steps;
    acc.evolve_ms += es.elapsed_ms;
    acc.timed_kernel_ms += es.timed_kernel_ms;
    acc.timed_kernel_launches += es.timed_kernel_launches;
    acc.loops += es.loops;
    acc.passed += es.passed;
    acc.batches += 1;
    for (size_t i = 0; i < b.regs.size(); ++i)
      log_region(b.regs[i], b.steps[i], b.ps[i], batch_id, es.elapsed_ms);
    batch_id++;
    return SEMIPAR_OK;
  }

  // Per-region event and loop lists into the caller's buffers, and the stats.
  int collect(const semipar_tiling* tt, const semipar_sched_params* pp, semipar_sched_stats* st,
              std::chrono::steady_clock::time_point t0) {
    const int nr = tt->n_regions;
    int64_t ne = 0;
    std::vector<int64_t> eoff((size_t)nr + 1, 0);
    for (int r = 0; r < nr; ++r) {
      eoff[r] = ne;
      if (pp->events) pp->events_off[r] = ne;
      ne += ev[r].size();
    }
    eoff[nr] = ne;
    if (pp->events) {
      pp->events_off[nr] = ne;
      // the copies into the caller's list, split over a few host threads by region
      auto part = [&](int r0, int r1) {
        for (int r = r0; r < r1; ++r) {
          const int64_t fit =
              std::max<int64_t>(0, std::min<int64_t>(eoff[r + 1], pp->events_cap) - eoff[r]);
          if (fit > 0) memcpy(pp->events + eoff[r], ev[r].data(), sizeof(semipar_event) * fit);
        }
      };
      const int nt = (int)std::min<int64_t>(8, std::max<int64_t>(1, ne / (1 << 16)));
      if (nt <= 1) {
        part(0, nr);
      } else {
        std::vector<std::thread> th;
        int r0 = 0;
        for (int k = 1; k <= nt; ++k) {
          // region boundary nearest to k / nt of the events
          int r1 = r0;
          while (r1 < nr && (k == nt || eoff[r1] < ne * k / nt)) ++r1;
          th.emplace_back(part, r0, r1);
          r0 = r1;
        }
        for (auto& x : th) x.join();
      }
    }
    acc.events = ne;
    int64_t nl = 0;
    for (int r = 0; r < nr; ++r) {
      const int64_t m = lp[r].size();
      if (pp->loops) {
        pp->loops_off[r] = nl;
        const int64_t fit = std::max<int64_t>(0, std::min(m, pp->loops_cap - nl));
        if (fit > 0) memcpy(pp->loops + nl, lp[r].data(), sizeof(semipar_loop) * fit);
      }
      nl += m;
    }
    if (pp->loops) pp->loops_off[nr] = nl;
    acc.makespan_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = acc;
    return SEMIPAR_OK;
  }

  // Ready regions into batches: longest predicted first (steps from the cost model, else
  // points), cut into batches of at most batch_points points, or into equal shares of
  // the predicted point-steps (PACK_WORK); each batch carries its predicted device time.
  std::vector<Batch> cut(std::vector<int32_t> live) {
    if (p->evolve.persistent) {
      // small regions go to batches of their own, which persistent workgroups evolve
      std::vector<int32_t> small, large;
      for (int32_t r : live)
        (t->surfaces[r].n <= SEMIPAR_PERSISTENT_MAX ? small : large).push_back(r);
      if (!small.empty() && !large.empty()) {
        std::vector<Batch> a = cut_some(large), b = cut_some(small);
        for (Batch& x : b) a.push_back(std::move(x));
        return a;
      }
    }
    return cut_some(live);
  }

  std::vector<Batch> cut_some(std::vector<int32_t> live) {
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
    return bs;
  }


  // Batched policy, dependency driven. The ready queue lives on the device
  // (k_dag_release); the host takes the regions that have become ready, packs them into
  // batches and hands those to idle lanes, longest predicted first. A region's
  // successors are released when its own batch has finished, not when a whole wave
  // has. A batch's results are taken on its lane as soon as it has evolved (harvest);
  // the batch regions are released, and the batches numbered in the order they were
  // formed, after the last one, since releasing device memory waits for the device.
  int run_dynamic() {
    const int nr = t->n_regions;
    const int lanes = std::max(1, p->lanes);
    std::vector<int32_t> hp((size_t)nr, 0), hoff((size_t)nr + 1, 0), hs;
    std::vector<uint8_t> hempty((size_t)nr, 0);
    for (int r = 0; r < nr; ++r) {
      hp[r] = t->n_pred ? t->n_pred[r] : 0;
      hempty[r] = t->surfaces[r].n == 0 ? 1 : 0;
    }
    if (t->n_pred) {
      for (int r = 0; r <= nr; ++r) hoff[r] = t->succ_off[r] - t->succ_off[0];
      hs.assign(t->succ + t->succ_off[0], t->succ + t->succ_off[nr]);
    }
    DagDev D;
    const size_t m = std::max<size_t>(hs.size(), 1);
    hipError_t ae = hipSuccess;
    if ((ae = hipMalloc(&D.pending, sizeof(int32_t) * std::max(nr, 1))) != hipSuccess ||
        (ae = hipMalloc(&D.succ_off, sizeof(int32_t) * (nr + 1))) != hipSuccess ||
        (ae = hipMalloc(&D.succ, sizeof(int32_t) * m)) != hipSuccess ||
        (ae = hipMalloc(&D.ring, sizeof(int32_t) * std::max(nr, 1))) != hipSuccess ||
        (ae = hipMalloc(&D.ctr, sizeof(int32_t) * 2)) != hipSuccess ||
        (ae = hipMalloc(&D.work, sizeof(int32_t) * std::max(nr, 1))) != hipSuccess ||
        (ae = hipMalloc(&D.fin, sizeof(int32_t) * std::max(nr, 1))) != hipSuccess ||
        (ae = hipMalloc(&D.empty, std::max(nr, 1))) != hipSuccess) {
      char msg[160];
      snprintf(msg, sizeof(msg), "schedule_regions: device allocation of the ready queue failed: %s",
               hipGetErrorString(ae));
      spi::set_error(msg);
      return ae == hipErrorOutOfMemory ? SEMIPAR_E_OOM : SEMIPAR_E_HIP;
    }
    std::vector<hipStream_t> ls((size_t)lanes, nullptr);
    std::vector<semipar_point_rec*> stage((size_t)lanes, nullptr);  // host output staging
    std::vector<int64_t> stage_cap((size_t)lanes, 0);
    hipStream_t ms = nullptr;  // the queue's kernels and reads, in order
    hipEvent_t ready_ev = nullptr;
    std::deque<Batch> bs;
    auto cleanup = [&]() {
      for (Batch& b : bs)
        if (b.reg) {
          region_destroy(b.reg);
          b.reg = nullptr;
        }
      for (semipar_point_rec* x : stage)
        if (x) (void)hipFree(x);
      for (hipStream_t x : ls)
        if (x) (void)hipStreamDestroy(x);
      if (ms) (void)hipStreamDestroy(ms);
      if (ready_ev) (void)hipEventDestroy(ready_ev);
    };
    int rc = SEMIPAR_OK;
    hipError_t he = hipStreamCreateWithFlags(&ms, hipStreamNonBlocking);
    if (he != hipSuccess) rc = hip_err(he, "queue stream");
    for (int l = 0; l < lanes && rc == SEMIPAR_OK; ++l)
      if ((he = hipStreamCreateWithFlags(&ls[l], hipStreamNonBlocking)) != hipSuccess)
        rc = hip_err(he, "lane stream");
    if (rc == SEMIPAR_OK && t->stream) {
      // device-resident surfaces may still be in flight on the caller's stream
      if ((he = hipEventCreateWithFlags(&ready_ev, hipEventDisableTiming)) != hipSuccess ||
          (he = hipEventRecord(ready_ev, (hipStream_t)t->stream)) != hipSuccess)
        rc = hip_err(he, "event on the caller's stream");
      for (int l = 0; l < lanes && rc == SEMIPAR_OK; ++l)
        if ((he = hipStreamWaitEvent(ls[l], ready_ev, 0)) != hipSuccess)
          rc = hip_err(he, "lane wait");
    }
    const int32_t zero2[2] = {0, 0};
    if (rc == SEMIPAR_OK &&
        ((he = hipMemcpyAsync(D.pending, hp.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice,
                              ms)) != hipSuccess ||
         (he = hipMemcpyAsync(D.succ_off, hoff.data(), sizeof(int32_t) * (nr + 1),
                              hipMemcpyHostToDevice, ms)) != hipSuccess ||
         (!hs.empty() && (he = hipMemcpyAsync(D.succ, hs.data(), sizeof(int32_t) * hs.size(),
                                              hipMemcpyHostToDevice, ms)) != hipSuccess) ||
         (he = hipMemcpyAsync(D.empty, hempty.data(), (size_t)nr, hipMemcpyHostToDevice, ms)) !=
             hipSuccess ||
         (he = hipMemcpyAsync(D.ctr, zero2, sizeof(zero2), hipMemcpyHostToDevice, ms)) !=
             hipSuccess))
      rc = hip_err(he, "queue upload");
    if (rc == SEMIPAR_OK) {
      (void)hipGetLastError();  // only this launch's error counts below
      k_dag_release<<<1, DAG_NT, 0, ms>>>(nullptr, 0, 1, nr, D.pending, D.succ_off, D.succ,
                                          D.empty, D.ring, D.ctr, D.work);
      if ((he = hipGetLastError()) != hipSuccess) rc = hip_err(he, "k_dag_release (seed)");
    }
    // regions that have entered the ring since the last read: empty ones are only
    // noted, the others wait for a batch
    std::vector<int32_t> host_ring((size_t)std::max(nr, 1));
    int32_t consumed = 0;
    auto drain = [&](std::vector<int32_t>& live) -> int {
      int32_t tail = 0;
      hipError_t e = hipMemcpyAsync(&tail, D.ctr, sizeof(int32_t), hipMemcpyDeviceToHost, ms);
      if (e == hipSuccess) e = hipStreamSynchronize(ms);
      if (e != hipSuccess) return hip_err(e, "ready-ring count read");
      if (tail < consumed || tail > nr) {
        spi::set_error("schedule_regions: the ready ring holds an impossible count");
        return SEMIPAR_E_HIP;
      }
      if (tail > consumed) {
        e = hipMemcpyAsync(host_ring.data() + consumed, D.ring + consumed,
                           sizeof(int32_t) * (tail - consumed), hipMemcpyDeviceToHost, ms);
        if (e == hipSuccess) e = hipStreamSynchronize(ms);
        if (e != hipSuccess) return hip_err(e, "ready-ring read");
      }
      for (int32_t i = consumed; i < tail; ++i) {
        const int32_t r = host_ring[i];
        acc.regions += 1;
        if (hempty[r]) {
          acc.empty_regions += 1;
          if (p->out_off)
            for (int f = 0; f < 4; ++f) p->out_off[4 * r + f] = slab[r].base;
          log_region(r, 0, 0, -1, 0.0);
        } else {
          live.push_back(r);
        }
      }
      consumed = tail;
      return SEMIPAR_OK;
    };
    std::mutex mu;
    std::condition_variable cv_lane, cv_mgr;
    std::vector<size_t> jobq;  // batches waiting for a lane, longest predicted last
    std::vector<size_t> done;  // batches finished since the manager last looked
    int running = 0;
    bool stop = false;
    auto dispatch = [&](std::vector<int32_t>& live) {
      if (live.empty()) return;
      std::vector<Batch> nb = cut(live);
      live.clear();
      std::lock_guard<std::mutex> lk(mu);
      for (Batch& b : nb) {
        bs.push_back(std::move(b));
        jobq.push_back(bs.size() - 1);
      }
      std::stable_sort(jobq.begin(), jobq.end(),
                       [&](size_t a, size_t b) { return bs[a].cost < bs[b].cost; });
    };
    std::vector<int32_t> live;
    if (rc == SEMIPAR_OK) rc = drain(live);
    if (rc == SEMIPAR_OK) dispatch(live);
    // The worker pool (Section "Implementation"): lanes take batches from jobq. With
    // lane_sleep_ms > 0 the pool is elastic as the paper's: a lane with nothing to do
    // sleeps, is woken by new batches, and exits once it has slept lane_sleep_ms; when
    // batches have waited lane_submit_ms for a lane, the manager starts lanes again (up to
    // `lanes`, in free slots). Lifetimes and busy times are summed for the stats.
    const double sleep_ms = p->lane_sleep_ms, submit_ms = p->lane_submit_ms;
    const bool elastic = sleep_ms > 0.0;
    const auto tb0 = std::chrono::steady_clock::now();
    auto now_ms = [&]() {
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb0)
          .count();
    };
    std::vector<std::thread> th((size_t)lanes);
    std::vector<char> alive((size_t)lanes, 0);
    int n_alive = 0;
    double held_ms = 0.0, busy_ms = 0.0;
    int64_t started = 0;
    auto lane_body = [&](int l, double t_start) {
      for (;;) {
        size_t i;
        {
          std::unique_lock<std::mutex> lk(mu);
          auto ready = [&] { return stop || !jobq.empty(); };
          bool got = true;
          if (elastic)
            got = cv_lane.wait_for(lk, std::chrono::duration<double, std::milli>(sleep_ms), ready);
          else
            cv_lane.wait(lk, ready);
          if (!got || jobq.empty()) {
            // slept with nothing to do, or the run is over: the lane exits (last use of mu)
            alive[l] = 0;
            --n_alive;
            held_ms += now_ms() - t_start;
            cv_mgr.notify_one();
            return;
          }
          i = jobq.back();
          jobq.pop_back();
          ++running;
        }
        const double tb = now_ms();
        Batch& b = bs[i];
        int brc = build_batch(b, ls[l]);
        if (brc == SEMIPAR_OK) brc = region_evolve(b.reg, &p->evolve, &b.es);
        if (brc == SEMIPAR_E_OVERFLOW && p->evolve.persistent) {
          // a step held more crossings than a persistent workgroup keeps: the
          // batch runs again from its surfaces on the step kernels
          region_destroy(b.reg);
          b.reg = nullptr;
          semipar_evolve_params e2 = p->evolve;
          e2.persistent = 0;
          brc = build_batch(b, ls[l]);
          if (brc == SEMIPAR_OK) brc = region_evolve(b.reg, &e2, &b.es);
        }
        if (brc == SEMIPAR_OK) brc = harvest(b, stage[l], stage_cap[l]);
        if (brc != SEMIPAR_OK) b.msg = semipar_last_error();
        {
          std::lock_guard<std::mutex> lk(mu);
          b.rc = brc;
          done.push_back(i);
          --running;
          busy_ms += now_ms() - tb;
        }
        cv_mgr.notify_one();
      }
    };
    auto start_lane = [&](int l) {  // with mu held; slot l's previous lane has returned
      if (th[(size_t)l].joinable()) th[(size_t)l].join();
      alive[(size_t)l] = 1;
      ++n_alive;
      ++started;
      th[(size_t)l] = std::thread(lane_body, l, now_ms());
    };
    if (rc == SEMIPAR_OK) {
      std::lock_guard<std::mutex> lk(mu);
      for (int l = 0; l < lanes; ++l) start_lane(l);
    }
    double waiting_since = -1.0;  // batches waiting for a lane since then (elastic pool)
    cv_lane.notify_all();
    std::vector<int32_t> fin;
    while (rc == SEMIPAR_OK) {
      std::vector<size_t> got;
      bool over = false;
      {
        std::unique_lock<std::mutex> lk(mu);
        auto ev = [&] { return !done.empty() || (running == 0 && jobq.empty()); };
        if (elastic) {
          cv_mgr.wait_for(lk, std::chrono::duration<double, std::milli>(
                                  std::max(0.05, std::min(submit_ms, sleep_ms) / 4)), ev);
          // batches waiting for more lanes than are idle: start lanes once that has
          // lasted lane_submit_ms
          const int idle = n_alive - running;
          if ((int)jobq.size() > idle && n_alive < lanes) {
            if (waiting_since < 0.0) waiting_since = now_ms();
            if (now_ms() - waiting_since >= submit_ms) {
              int want = (int)jobq.size() - idle;
              for (int l = 0; l < lanes && want > 0; ++l)
                if (!alive[(size_t)l]) {
                  start_lane(l);
                  --want;
                }
              waiting_since = -1.0;
              cv_lane.notify_all();
            }
          } else {
            waiting_since = -1.0;
          }
        } else {
          cv_mgr.wait(lk, ev);
        }
        got.swap(done);
        over = got.empty() && running == 0 && jobq.empty();
      }
      if (over) break;  // nothing running, nothing waiting: every ready region ran
      if (got.empty()) continue;
      fin.clear();
      for (size_t i : got) {
        if (bs[i].rc != SEMIPAR_OK && rc == SEMIPAR_OK) {
          rc = bs[i].rc;
          spi::set_error(bs[i].msg.c_str());  // the lane's message, on the caller's thread
        }
        fin.insert(fin.end(), bs[i].regs.begin(), bs[i].regs.end());
      }
      if (rc != SEMIPAR_OK) break;
      if ((he = hipMemcpyAsync(D.fin, fin.data(), sizeof(int32_t) * fin.size(),
                               hipMemcpyHostToDevice, ms)) != hipSuccess) {
        rc = hip_err(he, "finished-region list upload");
        break;
      }
      (void)hipGetLastError();  // only this launch's error counts below
      k_dag_release<<<1, DAG_NT, 0, ms>>>(D.fin, (int)fin.size(), 0, nr, D.pending, D.succ_off,
                                          D.succ, D.empty, D.ring, D.ctr, D.work);
      if ((he = hipGetLastError()) != hipSuccess) rc = hip_err(he, "k_dag_release");
      if (rc == SEMIPAR_OK) rc = drain(live);
      if (rc == SEMIPAR_OK) dispatch(live);
      cv_lane.notify_all();
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      if (rc != SEMIPAR_OK) jobq.clear();
      stop = true;
    }
    cv_lane.notify_all();
    for (auto& x : th)
      if (x.joinable()) x.join();
    acc.lane_held_ms = held_ms;
    acc.lane_busy_ms = busy_ms;
    acc.lanes_started = started;
    if (rc == SEMIPAR_OK && consumed != nr) {
      spi::set_error("schedule_regions: the predecessor counts leave regions that never become ready");
      rc = SEMIPAR_E_ARG;
    }
    // results, batch by batch in the order they were formed
    for (size_t i = 0; i < bs.size() && rc == SEMIPAR_OK; ++i) rc = finish_batch(bs[i]);
    cleanup();
    return rc;
  }

  // plain policy: one wave of ready regions, one region at a time
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
    for (int32_t r : live) RCCHK_R(run_plain(r));
    return SEMIPAR_OK;
  }
};

}  // namespace

extern "C" {

int schedule_regions(const semipar_tiling* t, const semipar_sched_params* p,
                     semipar_sched_stats* st) {
  spi::begin_call();
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
  if (!(p->lane_sleep_ms >= 0.0 && p->lane_submit_ms >= 0.0)) return SEMIPAR_E_ARG;
  const double cf = p->evolve.cell_factor;
  if (!(cf == 0.0 || (cf >= 1.0 && cf <= 4.0))) return SEMIPAR_E_ARG;
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
  bool any_points = false;
  for (int r = 0; r < nr; ++r) any_points = any_points || t->surfaces[r].n > 0;
  if (p->policy == SEMIPAR_SCHED_BATCHED && any_points) {
    rc = R.run_dynamic();
    if (rc != SEMIPAR_OK) return rc;
    return R.collect(t, p, st, t0);
  }
  // plain policy (one region at a time), or nothing to simulate: wave by wave of ready
  // regions, counted on the host
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
  return R.collect(t, p, st, t0);
}

int semipar_region_features(const semipar_tiling* t, float* feat) {
  spi::begin_call();
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
