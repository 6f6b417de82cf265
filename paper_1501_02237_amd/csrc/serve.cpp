// Serving engine: continuous batching of degree requests on one device.
//
// A host engine thread owns a device arena of request slots.  Each slot holds
// one admitted request's point set, heights and 128-bit partial sum; they stay
// resident while the request's work units are drained.  The engine loop:
//   1. takes newly submitted requests and runs their host prologue
//      (rank, components, kernel points, bounds);
//   2. admits waiting requests in arrival order while a slot is free and the
//      device-memory budget allows (slot bytes + the request's work units);
//   3. builds one step: a bounded quantum of work units taken round-robin
//      from every active request, so that new arrivals join the next step and
//      small requests are not stuck behind large ones;
//   4. runs the step (one enumeration launch over the mixed list) and reads
//      the partial sums of the slots back;
//   5. retires requests whose work units are all done (a tied lifting is
//      redrawn in place and its units re-queued) and wakes their waiters.
// Results equal those of bdeg_degree for the same input: the same host
// prologue, the same lifting stream (system index 0, attempt a) and the same
// exact device arithmetic.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.hpp"
#include "runtime.hpp"

using namespace bdeg;

namespace {

constexpr int SLOT_PTS = 64 * BDEG_MAX_K; // int32 coordinates per slot
constexpr int SLOT_HTS = 64;              // int64 heights per slot
constexpr size_t SLOT_BYTES = SLOT_PTS * 4 + SLOT_HTS * 8 + sizeof(SysAcc) + sizeof(SysDesc);
constexpr int MAX_SLOTS = 4096;
// One wavefront decides roughly 1-2e6 candidates per second (the device's
// throughput comes from thousands of wavefronts), so a step is many small
// units: about 2000 candidates each (a millisecond or two on one wavefront),
// a few tens of millions per step (a few milliseconds on the whole device).
constexpr uint32_t STEP_TILES_MAX = 32768;
constexpr uint64_t STEP_CANDIDATES = 24000000; // quantum of one step
constexpr uint64_t UNIT_COST = 2048;           // work-unit size cap for served requests

constexpr size_t LIGHT_LOAD = 8; // requests queued or running below which units are small
constexpr uint64_t LIGHT_UNIT_FLOOR = 256; // smallest unit under light load

// Work-unit size of a request.  Under light load (few requests queued or
// running) the request alone is spread over the resident wavefronts in units
// of at least LIGHT_UNIT_FLOOR candidates (below a plain solve's floor: here
// latency counts, not throughput), so that a small request is not one
// wavefront's work; otherwise UNIT_COST, so that a step of a full device
// carries its whole quantum within the step's unit limit.
uint64_t request_unit_cost(int N, int k, bool light) {
  if (!light) return UNIT_COST;
  return std::min<uint64_t>(UNIT_COST, choose_max_cost(binom_u64(N, k + 1), default_waves(k, k, 4), LIGHT_UNIT_FLOOR));
}
constexpr size_t PROLOGUE_THREADS = 8;         // host prologue workers for a burst of submissions

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  std::vector<int64_t> A;
  int m = 0, n = 0, bits = 20;
  uint64_t seed = 0;
  bdeg_result res{};
  HostSys hs;
  bool need_dev = false;
  bool dense = false; // runs in the lane-dense kernel
  int state = 0; // 0 queued, 1 waiting admission, 2 active, 3 done, 4 taken
  int slot = -1;
  std::vector<Tile> tiles;
  size_t next = 0;       // next unit to issue
  size_t bytes = 0;      // device budget charged while active
  Clock::time_point t_submit, t_done;
};

} // namespace

struct bdeg_server {
  size_t budget = 0, used = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool closing = false;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request *> submitted;
  std::thread engine;
  int status = BDEG_OK;

  // engine-owned
  hipStream_t stream = nullptr;
  // one stream, counter block and join event per k: a step's work units are
  // grouped by k and each group runs the single-k kernel concurrently
  hipStream_t kstream[BDEG_MAX_K + 1] = {};
  hipEvent_t kdone[BDEG_MAX_K + 1] = {};
  hipEvent_t step_ready = nullptr;
  SysDesc *d_sys = nullptr;
  int32_t *d_pts = nullptr;
  int64_t *d_hts = nullptr;
  SysAcc *d_acc = nullptr;
  Tile *d_tiles = nullptr;
  DevCounters *d_cnt = nullptr;
  int32_t *d_list = nullptr;
  Tile *h_tiles = nullptr;  // pinned
  SysAcc *h_acc = nullptr;  // pinned
  int32_t *h_list = nullptr; // pinned
  DevCounters *h_cnt = nullptr; // pinned, one block per (k, kernel variant) of a step
  std::vector<SysDesc> h_sys;
  std::vector<int> free_slots;
  std::deque<Request *> waiting;
  std::vector<Request *> active;
  int max_slots = 0;

  void run();
  int setup_device();
  void release_device();
  bool admit(Request *r);
  void start_attempt(Request *r);
  void finish(Request *r, int status);
  bool light = true; // few requests queued or running (set before each admission round)
};

int bdeg_server::setup_device() {
  max_slots = (int)std::min<size_t>(MAX_SLOTS, std::max<size_t>(1, budget / SLOT_BYTES));
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return BDEG_E_DEVICE;
  if (hipMalloc((void **)&d_sys, max_slots * sizeof(SysDesc)) != hipSuccess ||
      hipMalloc((void **)&d_pts, (size_t)max_slots * SLOT_PTS * 4) != hipSuccess ||
      hipMalloc((void **)&d_hts, (size_t)max_slots * SLOT_HTS * 8) != hipSuccess ||
      hipMalloc((void **)&d_acc, max_slots * sizeof(SysAcc)) != hipSuccess ||
      hipMalloc((void **)&d_tiles, STEP_TILES_MAX * sizeof(Tile)) != hipSuccess ||
      hipMalloc((void **)&d_cnt, (BDEG_MAX_K + 1) * GROUP_SLOTS * sizeof(DevCounters)) != hipSuccess ||
      hipMalloc((void **)&d_list, max_slots * sizeof(int32_t)) != hipSuccess)
    return BDEG_E_NOMEM;
  if (hipHostMalloc((void **)&h_tiles, STEP_TILES_MAX * sizeof(Tile), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h_acc, max_slots * sizeof(SysAcc), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h_list, max_slots * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h_cnt, (BDEG_MAX_K + 1) * GROUP_SLOTS * sizeof(DevCounters), hipHostMallocDefault) !=
          hipSuccess)
    return BDEG_E_NOMEM;
  h_sys.assign(max_slots, SysDesc{});
  for (int s = max_slots - 1; s >= 0; s--) free_slots.push_back(s);
  if (hipEventCreateWithFlags(&step_ready, hipEventDisableTiming) != hipSuccess) return BDEG_E_DEVICE;
  for (int k = 1; k <= BDEG_MAX_K; k++)
    if (hipStreamCreateWithFlags(&kstream[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&kdone[k], hipEventDisableTiming) != hipSuccess)
      return BDEG_E_DEVICE;
  return BDEG_OK;
}

void bdeg_server::release_device() {
  if (stream) (void)hipStreamSynchronize(stream);
  if (d_sys) (void)hipFree(d_sys);
  if (d_pts) (void)hipFree(d_pts);
  if (d_hts) (void)hipFree(d_hts);
  if (d_acc) (void)hipFree(d_acc);
  if (d_tiles) (void)hipFree(d_tiles);
  if (d_cnt) (void)hipFree(d_cnt);
  if (d_list) (void)hipFree(d_list);
  if (h_tiles) (void)hipHostFree(h_tiles);
  if (h_acc) (void)hipHostFree(h_acc);
  if (h_list) (void)hipHostFree(h_list);
  if (h_cnt) (void)hipHostFree(h_cnt);
  for (int k = 1; k <= BDEG_MAX_K; k++) {
    if (kstream[k]) (void)hipStreamDestroy(kstream[k]);
    if (kdone[k]) (void)hipEventDestroy(kdone[k]);
  }
  if (step_ready) (void)hipEventDestroy(step_ready);
  if (stream) (void)hipStreamDestroy(stream);
  stream = nullptr;
}

void bdeg_server::finish(Request *r, int status) {
  if (r->state == 2) {
    free_slots.push_back(r->slot);
    used -= r->bytes;
  }
  r->res.status = status;
  r->t_done = Clock::now();
  // the result and the latency stay readable until close; the request's
  // matrix, points and work units are no longer needed
  std::vector<int64_t>().swap(r->A);
  std::vector<int32_t>().swap(r->hs.pts);
  std::vector<Tile>().swap(r->tiles);
  std::lock_guard<std::mutex> lk(mu);
  r->state = 3;
  cv_done.notify_all();
}

// (Re)start the device work of an active request for its current attempt:
// lifting key, heights, cleared partial sum, fresh work units.
void bdeg_server::start_attempt(Request *r) {
  SysDesc &d = h_sys[r->slot];
  d.N = r->hs.N;
  d.k = r->hs.k;
  d.pt_off = r->slot * SLOT_PTS;
  d.ht_off = r->slot * SLOT_HTS;
  d.lift_bits = r->hs.lift_bits;
  d.npad_log2 = npad_log2_for(d.N);
  d.lift_key = lift_key(r->hs.seed, 0u, r->hs.attempt); // the single-system stream
  d.seed = r->hs.seed;
  d.sys_index = 0;
  r->dense = dense_ok(r->hs.pts.data(), d.N, d.k, (1ull << d.lift_bits) - 1);
  d.flags = r->dense ? SYS_DENSE | SYS_SORTED : 0; // served whole
  (void)hipMemcpyAsync(d_sys + r->slot, &d, sizeof(SysDesc), hipMemcpyHostToDevice, stream);
  // units are taken round-robin across requests in small steps, so their
  // order within a request does not matter: no sort
  std::vector<TileC> tc;
  tiles_full(d.N, d.k, (uint32_t)r->slot, request_unit_cost(d.N, d.k, light), tc);
  r->tiles.resize(tc.size());
  for (size_t i = 0; i < tc.size(); i++) r->tiles[i] = tc[i].t;
  r->next = 0;
}

// Device bytes charged to a request while it is active: its slot (points,
// heights, descriptor, partial sum) and its share of the step's unit buffer.
bool bdeg_server::admit(Request *r) {
  const uint64_t cand = binom_u64(r->hs.N, r->hs.k + 1);
  const size_t units_est = (size_t)(cand / request_unit_cost(r->hs.N, r->hs.k, light) + r->hs.N);
  const size_t need = SLOT_BYTES + std::min<size_t>(units_est, STEP_TILES_MAX) * sizeof(Tile);
  if (free_slots.empty() || used + need > budget) return false;
  r->slot = free_slots.back();
  free_slots.pop_back();
  r->bytes = need;
  used += need;
  r->state = 2;
  (void)hipMemcpyAsync(d_pts + (size_t)r->slot * SLOT_PTS, r->hs.pts.data(), r->hs.pts.size() * 4,
                       hipMemcpyHostToDevice, stream);
  start_attempt(r);
  return true;
}

void bdeg_server::run() {
  int st;
  Device *D = device_get(&st);
  if (!D) {
    status = st;
  } else {
    (void)D;
    status = setup_device();
  }
  std::vector<Request *> fresh, relift;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return closing || !submitted.empty() || !active.empty() || !waiting.empty(); });
      if (closing && submitted.empty() && active.empty() && waiting.empty()) break;
      fresh.assign(submitted.begin(), submitted.end());
      submitted.clear();
    }
    // 1. host prologue (a burst is split over worker threads; results are
    //    then queued in arrival order)
    {
      auto work = [&](size_t lo, size_t hi) {
        for (size_t i = lo; i < hi; i++) {
          Request *r = fresh[i];
          r->need_dev = prepare_one(r->A.data(), r->m, r->n, r->seed, r->bits, 0, r->res, r->hs);
        }
      };
      const size_t nf = fresh.size();
      const size_t nt = nf >= 32 ? std::min<size_t>(PROLOGUE_THREADS, nf / 16) : 1;
      std::vector<std::thread> th;
      for (size_t t = 1; t < nt; t++) th.emplace_back(work, nf * t / nt, nf * (t + 1) / nt);
      work(0, nf / nt);
      for (auto &x : th) x.join();
    }
    for (Request *r : fresh) {
      if (!r->need_dev) {
        finish(r, r->res.status);
        continue;
      }
      if (status != BDEG_OK) {
        finish(r, status);
        continue;
      }
      r->state = 1;
      waiting.push_back(r);
    }
    fresh.clear();
    // 2. admission in arrival order (relift still holds requests whose tied
    //    lifting was redrawn at the end of the previous step)
    light = active.size() + waiting.size() < LIGHT_LOAD;
    while (!waiting.empty() && admit(waiting.front())) {
      relift.push_back(waiting.front());
      waiting.pop_front();
      active.push_back(relift.back());
    }
    if (active.empty()) {
      // nothing runs, so the head of the queue can never fit the budget
      if (!waiting.empty()) {
        finish(waiting.front(), BDEG_E_NOMEM);
        waiting.pop_front();
      }
      continue;
    }
    // heights and cleared partial sums for newly admitted and redrawn requests;
    // h_list is rewritten only after the step's stream synchronisation below
    if (!relift.empty()) {
      for (size_t i = 0; i < relift.size(); i++) h_list[i] = relift[i]->slot;
      (void)hipMemcpyAsync(d_list, h_list, relift.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
      launch_lift(stream, d_sys, d_list, (int)relift.size(), d_hts);
      launch_clear_list(stream, d_acc, d_list, (int)relift.size());
      relift.clear();
    }
    // 3. one step: round-robin quanta over the active requests, then the
    //    units grouped by k (one single-k launch per group, concurrently)
    // units grouped by (k, kernel variant): index k * GROUP_SLOTS + slot
    constexpr int NB = (BDEG_MAX_K + 1) * GROUP_SLOTS;
    std::vector<Tile> byk[NB];
    uint32_t nt = 0;
    uint64_t budget_c = STEP_CANDIDATES;
    bool progress = true;
    while (progress && nt < STEP_TILES_MAX && budget_c > 0) {
      progress = false;
      for (Request *r : active) {
        if (r->next >= r->tiles.size() || nt >= STEP_TILES_MAX) continue;
        const Tile &t = r->tiles[r->next++];
        byk[r->hs.k * GROUP_SLOTS + group_slot(single_group(r->hs.N), r->dense)].push_back(t);
        nt++;
        uint64_t s0, e0;
        tile_interval(t, r->hs.k, &s0, &e0);
        budget_c = budget_c > (e0 - s0) ? budget_c - (e0 - s0) : 0;
        progress = true;
        if (budget_c == 0) break;
      }
    }
    int rc = BDEG_OK;
    if (nt > 0) {
      uint32_t off = 0, start[NB];
      for (int b = 0; b < NB; b++) {
        start[b] = off;
        if (!byk[b].empty()) memcpy(h_tiles + off, byk[b].data(), byk[b].size() * sizeof(Tile));
        off += (uint32_t)byk[b].size();
      }
      if (hipMemcpyAsync(d_tiles, h_tiles, nt * sizeof(Tile), hipMemcpyHostToDevice, stream) != hipSuccess)
        rc = BDEG_E_DEVICE;
      if (!rc) rc = launch_clear(stream, nullptr, 0, d_cnt, NB);
      int groups = 0;
      for (int b = 0; b < NB; b++) groups += !byk[b].empty();
      if (!rc && groups == 1) { // one group: launch it on the engine stream itself
        for (int b = 0; b < NB && !rc; b++) {
          if (byk[b].empty()) continue;
          LaunchShape shape;
          shape.single = b % GROUP_SLOTS == group_slot(true, false);
          shape.dense = b % GROUP_SLOTS == group_slot(false, true);
          rc = launch_enumerate(stream, d_sys, d_pts, d_hts, d_tiles + start[b], (uint32_t)byk[b].size(), d_acc,
                                d_cnt + b, b / GROUP_SLOTS, b / GROUP_SLOTS, shape);
        }
      }
      if (!rc && groups > 1 && hipEventRecord(step_ready, stream) != hipSuccess) rc = BDEG_E_DEVICE;
      for (int k = 1; k <= BDEG_MAX_K && !rc && groups > 1; k++) {
        bool any = false;
        for (int gs = 0; gs < GROUP_SLOTS; gs++) any |= !byk[k * GROUP_SLOTS + gs].empty();
        if (!any) continue;
        if (hipStreamWaitEvent(kstream[k], step_ready, 0) != hipSuccess) {
          rc = BDEG_E_DEVICE;
          break;
        }
        for (int gs = 0; gs < GROUP_SLOTS && !rc; gs++) {
          const int b = k * GROUP_SLOTS + gs;
          if (byk[b].empty()) continue;
          LaunchShape shape;
          shape.single = gs == group_slot(true, false);
          shape.dense = gs == group_slot(false, true);
          rc = launch_enumerate(kstream[k], d_sys, d_pts, d_hts, d_tiles + start[b], (uint32_t)byk[b].size(), d_acc,
                                d_cnt + b, k, k, shape);
        }
        if (!rc && (hipEventRecord(kdone[k], kstream[k]) != hipSuccess ||
                    hipStreamWaitEvent(stream, kdone[k], 0) != hipSuccess))
          rc = BDEG_E_DEVICE;
      }
    }
    // 4. partial sums of all active slots
    constexpr size_t CNT_BYTES = (BDEG_MAX_K + 1) * GROUP_SLOTS * sizeof(DevCounters);
    int used = 0; // slots up to the highest one in use
    for (Request *r : active) used = std::max(used, r->slot + 1);
    if (!rc && hipMemcpyAsync(h_acc, d_acc, used * sizeof(SysAcc), hipMemcpyDeviceToHost, stream) != hipSuccess)
      rc = BDEG_E_DEVICE;
    if (!rc && hipMemcpyAsync(h_cnt, d_cnt, CNT_BYTES, hipMemcpyDeviceToHost, stream) != hipSuccess)
      rc = BDEG_E_DEVICE;
    if (!rc && hipStreamSynchronize(stream) != hipSuccess) rc = BDEG_E_DEVICE;
    for (int b = 0; b < (BDEG_MAX_K + 1) * GROUP_SLOTS && !rc; b++)
      if (!byk[b].empty() && h_cnt[b].error) rc = BDEG_E_DEVICE;
    // 5. retire finished requests, relift tied ones
    std::vector<Request *> still;
    for (Request *r : active) {
      if (rc) {
        finish(r, rc);
        continue;
      }
      if (r->next < r->tiles.size()) {
        still.push_back(r);
        continue;
      }
      const SysAcc &a = h_acc[r->slot];
      r->res.attempts = (int32_t)r->hs.attempt + 1;
      if (a.tie) {
        if (r->hs.attempt + 1 >= BDEG_MAX_ATTEMPTS) {
          finish(r, BDEG_E_TIE);
          continue;
        }
        r->hs.attempt++;
        start_attempt(r);
        relift.push_back(r);
        still.push_back(r);
        continue;
      }
      r->res.nvol = bdeg_u128{a.lo, a.hi};
      r->res.cells = a.cells;
      finish(r, BDEG_OK);
    }
    active.swap(still);
  }
  release_device();
}

extern "C" {

int bdeg_serve_open(size_t device_mem_budget, bdeg_server **out) {
  if (!out || device_mem_budget < SLOT_BYTES) return BDEG_E_ARG;
  int st;
  if (!device_get(&st)) return st;
  bdeg_server *s = new bdeg_server();
  s->budget = device_mem_budget;
  s->engine = std::thread([s] { s->run(); });
  *out = s;
  return BDEG_OK;
}

int bdeg_serve_submit(bdeg_server *s, const int64_t *A, int32_t m, int32_t n, uint64_t seed, int32_t lift_bits,
                      uint64_t *ticket) {
  if (!s || !A || !ticket || m < 1 || n < 1 || n > BDEG_MAX_N) return BDEG_E_ARG;
  auto r = std::make_unique<Request>();
  r->A.assign(A, A + (size_t)m * n);
  r->m = m;
  r->n = n;
  r->seed = seed;
  r->bits = lift_bits;
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->closing) return BDEG_E_STATE;
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->submitted.push_back(r.get());
  s->reqs.emplace(r->ticket, std::move(r));
  s->cv_work.notify_one();
  return BDEG_OK;
}

static int take(bdeg_server *s, uint64_t ticket, bdeg_result *out, bool block) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->state == 4) return BDEG_E_STATE;
  Request *r = it->second.get();
  if (block)
    s->cv_done.wait(lk, [&] { return r->state == 3; });
  else if (r->state != 3)
    return BDEG_PENDING;
  *out = r->res;
  r->state = 4;
  return r->res.status;
}

int bdeg_serve_poll(bdeg_server *s, uint64_t ticket, bdeg_result *out) {
  if (!s || !out) return BDEG_E_ARG;
  return take(s, ticket, out, false);
}

int bdeg_serve_wait(bdeg_server *s, uint64_t ticket, bdeg_result *out) {
  if (!s || !out) return BDEG_E_ARG;
  return take(s, ticket, out, true);
}

int bdeg_serve_latency(bdeg_server *s, uint64_t ticket, uint64_t *submit_to_done_ns) {
  if (!s || !submit_to_done_ns) return BDEG_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return BDEG_E_STATE;
  Request *r = it->second.get();
  if (r->state < 3) return BDEG_PENDING;
  *submit_to_done_ns =
      (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(r->t_done - r->t_submit).count();
  return BDEG_OK;
}

int bdeg_serve_close(bdeg_server *s) {
  if (!s) return BDEG_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->closing = true;
    s->cv_work.notify_all();
  }
  if (s->engine.joinable()) s->engine.join();
  delete s;
  return BDEG_OK;
}

} // extern "C"
