// Multi-query engine: many adaptive runs (Algorithm 1 of Borassi & Natale), on one
// graph or many, share sampler launches and hit reductions.
//
// Every query keeps the schedule of a single run -- alpha pilot samples (phase 0),
// computeDelta (Algorithm 2), then main-phase samples (phase 1) with the stopping
// rule evaluated after every check interval of B samples -- and its result is exactly
// the single run's: sample ids, check points and the counts entering each check are
// the same, only the launches that carry them differ.
//
// One engine "tick" is one sampler launch.  It holds, for every active query, its
// next pilot samples and/or its next check intervals, laid out interval-major
// ("layers": layer j holds the j-th interval of every query that has one), so that a
// hit reduction per layer followed by a snapshot per layer gives each query the
// counts of exactly the samples up to each of its check points.  The node ids of a
// query live at a fixed offset in a shared counter pool (tile-aligned), so one
// reduction serves all queries of a layer.  Snapshots are the per-group maxima of
// the counts (all-nodes task; group = nodes with equal (L_l, L_u), kept current by
// the reduction itself) or the counts (top-k task).  A query's main phase starts once
// its computeDelta has run (its groups are then known); that runs as a task beside the
// engine thread, and until it is done other queries keep the device busy.
//
// While tick t runs on the GPU the host evaluates tick t-1's checks.  A query that
// stops has samples past its stopping point in flight: their hits are subtracted
// again before its counters are read, as in the single run.
//
// Two lanes of ticks run side by side, each with its own streams, sampler slots and
// reduction scratch: lane 0 for most graphs, lane 1 for high-diameter graphs whose
// samples all take the (slow) wide-count kernel, so that those never hold up the
// queries of lane 0.  Lane 1's running tick is polled, never waited on.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <future>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "kad_internal.h"
#include "kad_stats.h"

namespace kad {
namespace {

using clk = std::chrono::steady_clock;
double secs(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

constexpr uint32_t POOL_TILES = MAX_HIT_TILES_PUBLIC;                 // counter pool tiles
constexpr uint64_t POOL_IDS = (uint64_t)POOL_TILES * HIT_TILE_IDS;    // 2^25 node ids
constexpr uint32_t TICK_SAMPLES = 1u << 18;    // samples per engine launch, at most
constexpr uint64_t TICK_PATH_BYTES = 1ull << 30;  // path buffer of one launch, at most
constexpr uint32_t MAX_LAYERS = 64;            // check intervals of one query per launch
constexpr uint32_t MAX_PIECES = 1u << 16;      // segments of one launch
// Buffers of a running engine are sized once (or grow by doubling, their old storage
// released only while nothing runs): freeing device memory waits for the whole
// device, which would stall one lane behind the other.

enum class QState { Queued, Pilot, Main, Final, Done };
// Pilot: pilot samples; PilotLast: the last ones (snapshot = count0, then the
// counters restart); Main: a check interval, snapshot = group maxima (all-nodes) or
// counts (MainFull, top-k).
enum class Kind : uint8_t { Pilot, PilotLast, MainFull, Main };

struct Query {
  uint64_t ticket = 0;
  kad_graph *g = nullptr;
  kad_params p{};
  kad_result *direct = nullptr;  // kad_run_batch: per-node outputs go straight here
  QState st = QState::Queued;
  kad_status status = KAD_OK;
  std::string error;
  bool prepared = false;
  // schedule
  uint32_t n = 0, vd = 0, stride = 2;
  bool vd_exact = false;
  int ovc = 1;  // overflow_class of the graph
  int lane = 0;
  uint64_t omega = 0, alpha = 0, B = 0, K = 0;
  double eb = 0.001;
  // counter pool slice: node v of the query is pool id base() + v
  uint32_t tile0 = 0, ntiles = 0;
  uint64_t base() const { return (uint64_t)tile0 * HIT_TILE_IDS; }
  // progress
  uint64_t pilot_launched = 0, launched = 0, tau = 0;
  bool main_started = false, delta_ready = false, rule = false;
  double worst = 0.0;
  uint64_t arcs = 0, pilot_arcs = 0;
  int refs = 0;              // unprocessed ticks holding samples of this query
  uint64_t last_tick = ~0ull;  // the tick being built last added this query
  // statistics
  std::vector<uint64_t> count0;
  std::vector<double> lam_l, lam_u, L_l, L_u;
  std::unique_ptr<StopChecker> checker;
  double C = 0.0;
  // results: o_* point into the caller's arrays (direct) or into the vectors
  hipEvent_t final_ev = nullptr;
  std::vector<uint64_t> count;
  std::vector<double> bc, lo, hi;
  uint64_t *o_count = nullptr;
  double *o_bc = nullptr, *o_lo = nullptr, *o_hi = nullptr;
  std::vector<uint32_t> topk, rlo, rhi;
  // times
  clk::time_point t_submit, t_admit, t_pilot, t_delta, t_final, t_done;
  // computeDelta and the stopping check's setup, run beside the engine thread once the
  // pilot's counts are in; declared last: destroying it first waits for the task, which
  // writes the fields above
  std::future<void> delta_task;
  // the per-node outputs (Theorem 1 intervals, the top-k selection), computed beside the
  // engine thread once the final counts have landed
  std::future<void> out_task;
  ~Query() {
    if (final_ev) (void)hipEventDestroy(final_ev);
  }
};

struct Piece {
  Query *q;
  Kind kind;
  uint32_t begin, count;  // launch indices
  uint64_t first;         // first sample id
  uint64_t snap;          // snapshot offset (entries), pilots other than the last: none
};

struct Tick {
  OutSet out;
  DevBuf<uint32_t> wlist;  // samples left by the sampler to the wide-count kernel
  DevBuf<uint32_t> wlist2; // samples left by the first wide pass to the second
  // the recorded sampling chains of this tick's buffers, one per sampler block size and
  // wide-lane share (KAD_EXEC_GRAPH), and the descriptor they read
  BatchGraph chains[6];
  PinBuf<BatchDesc> h_bd;
  DevBuf<BatchDesc> d_bd;
  DevBuf<SampleSeg> d_segs;
  PinBuf<SampleSeg> h_segs;
  DevBuf<GatherDesc> d_gat;
  PinBuf<GatherDesc> h_gat;
  DevBuf<uint32_t> work;
  DevBuf<uint64_t> d_snap;
  PinBuf<uint64_t> h_snap;
  hipEvent_t sampled = nullptr;
  std::vector<hipEvent_t> layer_ev;
  std::vector<Piece> pieces;
  std::vector<Query *> queries;        // each query with samples in this tick, once
  std::vector<uint32_t> layer_piece;  // layer L = pieces [layer_piece[L], layer_piece[L+1])
  std::vector<uint32_t> layer_gat;    // its gather descriptors
  std::vector<uint32_t> layer_blocks; // and the gather's workgroups
  std::vector<uint64_t> layer_snap;   // and its snapshot entries
  uint32_t total = 0, stride = 2, layers = 0;
  uint32_t wide_wgs = 0;  // wide-count workgroups of the lane-1 launch (each fills a CU)
  uint64_t id = 0;
  bool in_flight = false;
  ~Tick() {
    if (sampled) (void)hipEventDestroy(sampled);
    for (auto e : layer_ev) (void)hipEventDestroy(e);
  }
};

struct Lane {
  Tick ticks[2];
  int cur = 0;                      // ticks[cur] is the next to fill
  hipStream_t s = nullptr, rs = nullptr;
  bool own_streams = false;
  DevBuf<uint32_t> bins, bin_count, tile_start, tile_fill;  // compact hit reduction
  uint64_t bins_cap = 0;
  uint32_t slot0 = 0, nslots = 0;   // sampler slots
  uint32_t wslot0 = 0, nwslots = 0; // wide-count slots (arena and slot arrays of that index)
  bool busy() const { return ticks[0].in_flight || ticks[1].in_flight; }
  // wide-count workgroups of the launches in flight
  uint32_t wide_in_flight() const {
    uint32_t w = 0;
    for (const Tick &t : ticks)
      if (t.in_flight) w = std::max(w, t.wide_wgs);
    return w;
  }
  HitScratch scratch() const {
    HitScratch h;
    h.bins = bins.p;
    h.cap = bins_cap;
    h.bin_count = bin_count.p;
    h.tile_start = tile_start.p;
    h.tile_fill = tile_fill.p;
    return h;
  }
};

}  // namespace

class Engine {
 public:
  explicit Engine(kad_ctx *c) : ctx_(c) {}
  ~Engine() {
    release_graveyard();
    for (Lane &L : lanes_) {
      if (L.s) (void)hipStreamSynchronize(L.s);
      if (L.rs) (void)hipStreamSynchronize(L.rs);
      if (L.own_streams) {
        (void)hipStreamDestroy(L.s);
        (void)hipStreamDestroy(L.rs);
      }
    }
  }
  kad_status init();
  void enqueue(Query *q) { queue_.push_back(q); }
  // A server's queries arrive at any time: the wide lane then always leaves three quarters
  // of the CUs to lane 0, not only while lane 0 has work.
  void set_serving(bool on) { serving_ = on; }
  bool busy() const {
    return !queue_.empty() || !active_.empty() || lanes_[0].busy() || lanes_[1].busy();
  }
  // One round: admit queued queries, launch a tick, evaluate the previous one, and
  // complete stopped queries whose counters have landed.
  kad_status step();
  std::vector<Query *> take_done() {
    std::vector<Query *> d;
    d.swap(done_);
    return d;
  }
  // Stop every admitted query (status KAD_ECANCELED; its in-flight samples drain
  // normally) and drop the queued ones.
  kad_status cancel_all();
  uint64_t ticks_launched() const { return ticks_launched_.load(); }
  uint64_t samples_launched() const { return samples_launched_.load(); }

 private:
  kad_status prepare(Query *q);
  kad_status admit();
  // Queries whose computeDelta task has finished: their group ids into the pool; they
  // enter the main phase.
  kad_status delta_done();
  kad_status build(int li, Tick &t);
  kad_status launch(Lane &L, Tick &t);
  kad_status process(Lane &L, Tick &t, Tick &other);
  kad_status stop_query(Query *q, Lane &L, Tick &t, size_t after_piece, Tick &other);
  kad_status finalize(bool block);
  kad_status reduce(const Lane &L, const Tick &t, uint32_t begin, uint32_t count, bool subtract);
  void release_tiles(Query *q);
  void finish_failed(Query *q, kad_status st, const std::string &msg);
  void layout();
  SlotState lane_slots(const Lane &L, bool wide) const;
  WideState lane_wide(const Lane &L) const;
  // the second wide pass's view of the lane's arena (slots 0 when the arena is small)
  WideState lane_wide2(const Lane &L) const;
  static bool tick_complete(const Tick &t);
  // Double a buffer's capacity (at least to n) without freeing: the old storage is
  // released by release_graveyard() once no lane runs.
  template <typename T>
  void grow(DevBuf<T> &b, size_t n) {
    if (b.p) grave_dev_.push_back(b.p);
    b.p = nullptr;
    const size_t want = std::max(n, 2 * b.n);
    b.n = 0;
    if (hipMalloc((void **)&b.p, want * sizeof(T)) == hipSuccess) b.n = want;
    else b.p = nullptr;
  }
  template <typename T>
  void grow(PinBuf<T> &b, size_t n) {
    if (b.p) grave_host_.push_back(b.p);
    b.p = nullptr;
    const size_t want = std::max(n, 2 * b.n);
    b.n = 0;
    if (hipHostMalloc((void **)&b.p, want * sizeof(T), hipHostMallocCoherent) == hipSuccess) b.n = want;
    else b.p = nullptr;
  }
  void release_graveyard() {
    for (void *p : grave_dev_) (void)hipFree(p);
    for (void *p : grave_host_) (void)hipHostFree(p);
    grave_dev_.clear();
    grave_host_.clear();
  }
  std::vector<void *> grave_dev_, grave_host_;

  kad_ctx *ctx_;
  DevBuf<uint64_t> count_pool_, gmax_pool_;
  PinBuf<uint64_t> final_pool_;  // host landing area of stopped queries' counters
  PinBuf<uint32_t> group_stage_; // pinned staging of group ids (a pageable copy would wait)
  DevBuf<uint32_t> group_pool_;
  std::vector<uint8_t> tile_used_;
  uint32_t tiles_hw_ = 0;  // reductions cover pool tiles [0, tiles_hw_)
  Lane lanes_[2];
  bool split_ = false;  // lane 1 in use
  uint64_t tick_id_ = 0;
  std::deque<Query *> queue_;
  std::vector<Query *> active_;
  std::vector<Query *> done_;
  size_t rr_ = 0;
  bool serving_ = false;
  bool delta_pending_ = false;  // a computeDelta task is still running
  bool out_pending_ = false;    // an outputs task is still running
  std::atomic<uint64_t> ticks_launched_{0}, samples_launched_{0};
};

kad_status Engine::init() {
  HIP_TRY(hipSetDevice(ctx_->device));
  HIP_TRY(count_pool_.ensure(POOL_IDS));
  HIP_TRY(gmax_pool_.ensure(POOL_IDS));
  HIP_TRY(group_pool_.ensure(POOL_IDS));
  HIP_TRY(final_pool_.ensure(POOL_IDS));
  HIP_TRY(group_stage_.ensure(POOL_IDS));
  HIP_TRY(hipMemsetAsync(count_pool_.p, 0, POOL_IDS * 8, ctx_->rstream));
  HIP_TRY(hipMemsetAsync(group_pool_.p, 0, POOL_IDS * 4, ctx_->rstream));
  lanes_[0].s = ctx_->stream;
  lanes_[0].rs = ctx_->rstream;
  HIP_TRY(hipStreamCreateWithFlags(&lanes_[1].s, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&lanes_[1].rs, hipStreamNonBlocking));
  lanes_[1].own_streams = true;
  for (Lane &L : lanes_) {
    HIP_TRY(L.bin_count.ensure(POOL_TILES));
    HIP_TRY(L.tile_start.ensure(POOL_TILES));
    HIP_TRY(L.tile_fill.ensure(POOL_TILES));
    HIP_TRY(hipMemsetAsync(L.bin_count.p, 0, POOL_TILES * 4, ctx_->rstream));
    HIP_TRY(hipMemsetAsync(L.tile_fill.p, 0, POOL_TILES * 4, ctx_->rstream));
    for (Tick &t : L.ticks) {
      HIP_TRY(t.work.ensure(WORK_WORDS));
      HIP_TRY(hipEventCreateWithFlags(&t.sampled, hipEventDisableTiming));
    }
  }
  HIP_TRY(hipStreamSynchronize(ctx_->rstream));
  tile_used_.assign(POOL_TILES, 0);
  layout();
  return KAD_OK;
}

// Lane 1 takes 3/4 of the wide-count slots; lane 0 keeps the rest of them for its
// overflowed samples and the sampler slots past all of them (all of them when the
// wide-count kernel has slots of its own).  Without enough slots, lane 0 alone serves
// everything.
void Engine::layout() {
  const uint32_t W = ctx_->w_slots ? std::min(ctx_->w_slots, wide_slot_count(ctx_)) : 0,
                 S = ctx_->slots;
  const uint32_t skip = ctx_->slot_hbits ? 0u : W;  // sampler slots the wide passes use
  Lane &a = lanes_[0], &b = lanes_[1];
  split_ = W >= 4 && S >= skip + 64;
  if (split_) {
    b.wslot0 = 0;
    b.nwslots = W * 3 / 4;
    b.slot0 = 0;
    b.nslots = 0;
    a.wslot0 = b.nwslots;
    a.nwslots = W - b.nwslots;
    a.slot0 = skip;
    a.nslots = S - skip;
  } else {
    a.wslot0 = 0;
    a.nwslots = W;
    a.slot0 = 0;
    a.nslots = S;
    b.nslots = b.nwslots = 0;
  }
}

SlotState Engine::lane_slots(const Lane &L, bool wide) const {
  SlotState st = wide ? wide_slot_view(ctx_, L.wslot0) : slot_view(ctx_, L.slot0);
  st.slots = wide ? L.nwslots : L.nslots;
  return st;
}

WideState Engine::lane_wide(const Lane &L) const {
  WideState w = wide_view(ctx_);
  w.arena += (size_t)L.wslot0 * w.arena_limbs;
  w.lv += (size_t)L.wslot0 * 2 * w.max_lev * 4;
  w.lbase += (size_t)L.wslot0 * 2 * w.max_lev;
  w.slots = L.nwslots;
  return w;
}

WideState Engine::lane_wide2(const Lane &L) const {
  WideState w = lane_wide(L);
  if (ctx_->w_slots2 == 0 || L.nwslots == 0) {
    w.slots = 0;
    return w;
  }
  const uint64_t total = (uint64_t)L.nwslots * w.arena_limbs;
  const uint64_t n2 = std::max<uint64_t>(1, total / ctx_->w_arena_limbs2);
  w.slots = (uint32_t)n2;
  w.arena_limbs = total / n2;
  return w;
}

bool Engine::tick_complete(const Tick &t) {
  if (hipEventQuery(t.out.copied) != hipSuccess) return false;
  return t.layers == 0 || hipEventQuery(t.layer_ev[t.layers - 1]) == hipSuccess;
}

void Engine::finish_failed(Query *q, kad_status st, const std::string &msg) {
  if (q->status == KAD_OK) {
    q->status = st;
    q->error = msg;
  }
}

kad_status Engine::prepare(Query *q) {
  q->prepared = true;
  const kad_params &p = q->p;
  q->n = q->g->n;
  if (q->n > POOL_IDS) {
    finish_failed(q, KAD_EINVAL, "the engine serves graphs of up to 2^25 nodes");
    return KAD_OK;
  }
  if (p.vd_override) {
    q->vd = p.vd_override;
  } else {
    kad_status s = graph_vd(q->g, &q->vd, &q->vd_exact);
    if (s) {
      finish_failed(q, s, kad_last_error());
      return KAD_OK;
    }
  }
  const double c = p.c > 0 ? p.c : 0.5;
  q->eb = p.balance_eps > 0 ? p.balance_eps : 0.001;
  q->omega = omega_of(p.epsilon, p.delta, q->vd, c);
  q->alpha = alpha_of(q->omega);
  q->B = p.check_interval ? p.check_interval : interval_of(q->omega);
  uint64_t K = p.kernel_batch ? p.kernel_batch : DEFAULT_BATCH;
  q->K = std::min<uint64_t>(std::max<uint64_t>(q->B, (K + q->B - 1) / q->B * q->B),
                            (uint64_t)q->B * MAX_LAYERS);
  q->stride = std::max<uint32_t>(q->vd, 2);
  q->ovc = overflow_class(q->g, q->vd, p.vd_override == 0);
  if (q->B > TICK_SAMPLES || (uint64_t)q->stride * 4 * q->B > TICK_PATH_BYTES)
    finish_failed(q, KAD_EINVAL, "check interval too large for the engine's launches");
  return KAD_OK;
}

void Engine::release_tiles(Query *q) {
  for (uint32_t t = q->tile0; t < q->tile0 + q->ntiles; ++t) tile_used_[t] = 0;
  q->ntiles = 0;
  tiles_hw_ = 0;
  for (uint32_t t = 0; t < POOL_TILES; ++t)
    if (tile_used_[t]) tiles_hw_ = t + 1;
}

// Admission: queries are taken in arrival order within each lane; a lane whose next
// query does not fit (counter pool, or slot memory that can only grow while nothing
// runs) waits without holding up the other lane.  Lane 1 (slow, high-diameter
// queries) may hold at most half of the counter pool.
kad_status Engine::admit() {
  bool blocked[2] = {false, false};
  uint32_t lane1_tiles = 0;
  for (const Query *q : active_)
    if (q->lane == 1) lane1_tiles += q->ntiles;
  for (size_t j = 0; j < queue_.size();) {
    Query *q = queue_[j];
    if (!q->prepared) {
      kad_status s = prepare(q);
      if (s) return s;
    }
    if (q->status != KAD_OK) {  // rejected before it touched the GPU
      queue_.erase(queue_.begin() + j);
      q->st = QState::Done;
      q->t_admit = q->t_pilot = q->t_delta = q->t_final = q->t_done = clk::now();
      done_.push_back(q);
      continue;
    }
    const int lane = split_ && q->ovc == 2 ? 1 : 0;
    if (blocked[lane]) {
      ++j;
      continue;
    }
    const uint32_t need = (uint32_t)((q->n + HIT_TILE_IDS - 1) / HIT_TILE_IDS);
    uint32_t start = POOL_TILES;
    if (lane == 0 || lane1_tiles + need <= POOL_TILES / 2) {
      for (uint32_t t = 0, run = 0; t < POOL_TILES; ++t) {  // first fit
        run = tile_used_[t] ? 0 : run + 1;
        if (run == need) {
          start = t + 1 - need;
          break;
        }
      }
    }
    if (start == POOL_TILES) {  // wait until running queries release counters
      blocked[lane] = true;
      ++j;
      continue;
    }
    const bool need_wide = !wide_fits(ctx_, q->g, q->ovc);
    if (q->n > ctx_->slot_n || need_wide) {
      if (lanes_[0].busy() || lanes_[1].busy()) break;  // grow only when idle
      for (Lane &L : lanes_) HIP_TRY(hipStreamSynchronize(L.rs));
      kad_status s = q->n > ctx_->slot_n ? ensure_slots(ctx_, q->n) : KAD_OK;
      if (!s) s = ensure_wide(ctx_, q->g, q->ovc);
      layout();
      if (s) finish_failed(q, s, kad_last_error());
      continue;  // looked at again with the new layout (or as failed)
    }
    q->lane = lane;
    if (lane == 1) lane1_tiles += need;
    for (uint32_t t = start; t < start + need; ++t) tile_used_[t] = 1;
    q->tile0 = start;
    q->ntiles = need;
    tiles_hw_ = std::max(tiles_hw_, start + need);
    // until computeDelta assigns groups, every node maps to the query's first
    // group-maximum entry
    HIP_TRY(launch_fill_u32(group_pool_.p + q->base(), q->n, (uint32_t)q->base(),
                            lanes_[q->lane].rs));
    if (!q->final_ev) HIP_TRY(hipEventCreateWithFlags(&q->final_ev, hipEventDisableTiming));
    q->st = QState::Pilot;
    q->t_admit = clk::now();
    active_.push_back(q);
    queue_.erase(queue_.begin() + j);
  }
  return KAD_OK;
}

kad_status Engine::build(int li, Tick &t) {
  t.pieces.clear();
  t.queries.clear();
  t.layer_piece.assign(1, 0);
  t.total = 0;
  t.stride = 2;
  t.layers = 0;
  t.id = ++tick_id_;
  std::vector<std::vector<Piece>> layer(MAX_LAYERS + 1);
  uint32_t total = 0, stride = 2;
  uint32_t npieces = 0;
  auto room = [&](const Query *q, uint64_t want) -> uint32_t {
    const uint32_t st = std::max(stride, q->stride);
    const uint64_t by_path = TICK_PATH_BYTES / (4ull * st);
    const uint64_t cap = std::min<uint64_t>(TICK_SAMPLES, by_path);
    if (npieces >= MAX_PIECES) return 0u;
    return total >= cap ? 0u : (uint32_t)std::min<uint64_t>(want, cap - total);
  };
  auto add = [&](Query *q, uint32_t L, Kind kind, uint32_t cnt, uint64_t first) {
    ++npieces;
    layer[L].push_back(Piece{q, kind, 0, cnt, first, ~0ull});
    total += cnt;
    stride = std::max(stride, q->stride);
    if (q->last_tick != t.id) {
      q->last_tick = t.id;
      q->refs++;
      t.queries.push_back(q);
    }
  };
  // With more than one query of the lane under way, none takes more than a quarter of a
  // tick: a tick lasts until its last sample, so one query's large batch would hold every
  // other query's next round trip (its check, then its next batch) for all that time.
  const size_t na = active_.size();
  uint32_t under_way = 0;
  for (const Query *q : active_)
    if (q->lane == li && q->status == KAD_OK && (q->st == QState::Pilot || q->st == QState::Main))
      ++under_way;
  const uint64_t per_query = under_way > 1 ? TICK_SAMPLES / 4 : TICK_SAMPLES;
  for (size_t j = 0; j < na; ++j) {
    Query *q = active_[(rr_ + j) % na];
    if (q->lane != li || q->status != KAD_OK || q->st == QState::Final) continue;
    if (q->st == QState::Pilot) {
      if (q->pilot_launched >= q->alpha) continue;  // waiting for computeDelta
      const uint32_t cnt = room(q, std::min<uint64_t>(q->alpha - q->pilot_launched,
                                                      std::min<uint64_t>(TICK_SAMPLES / 2, per_query)));
      if (cnt == 0) continue;
      const bool last = q->pilot_launched + cnt == q->alpha;
      add(q, 0, last ? Kind::PilotLast : Kind::Pilot, cnt, q->pilot_launched);
      q->pilot_launched += cnt;
      continue;
    }
    // main phase: the first batch is half the cap (in check intervals, at most K);
    // later ones are sized from the latest check
    if (q->st != QState::Main || q->launched >= q->omega) continue;
    uint64_t want;
    if (!q->main_started) {
      want = std::min<uint64_t>(q->omega, std::min<uint64_t>(q->K, std::max<uint64_t>(q->B, (q->omega / 2 + q->B - 1) / q->B * q->B)));
    } else {
      if (q->tau == 0) continue;  // first batch not yet checked
      const uint64_t ahead = q->launched - q->tau;
      double w;
      if (q->p.mode == KAD_ALL_NODES && q->worst > 0.0)
        w = (double)q->tau * q->worst - (double)q->launched;  // the bounds shrink about as 1/tau
      else
        w = (double)q->K - (double)ahead;
      if (w <= 0.0) {
        if (ahead > 0) continue;  // what is in flight is predicted to suffice
        w = (double)q->B;
      }
      want = (uint64_t)std::min<double>(std::ceil(w / (double)q->B), (double)(q->K / q->B)) * q->B;
    }
    want = std::min(want, per_query);  // at least one interval is still added
    const Kind kind = q->p.mode == KAD_TOPK ? Kind::MainFull : Kind::Main;
    for (uint32_t L = 0; L < MAX_LAYERS && want > 0 && q->launched < q->omega; ++L) {
      const uint32_t cnt = (uint32_t)std::min<uint64_t>(q->B, q->omega - q->launched);
      if (room(q, cnt) < cnt) break;
      add(q, L, kind, cnt, q->launched);
      q->launched += cnt;
      q->main_started = true;
      want = want > cnt ? want - cnt : 0;
    }
  }
  rr_ = na ? (rr_ + 1) % na : 0;
  uint32_t pos = 0;
  for (uint32_t L = 0; L <= MAX_LAYERS; ++L) {
    if (layer[L].empty()) break;
    for (Piece &pc : layer[L]) {
      pc.begin = pos;
      pos += pc.count;
      t.pieces.push_back(pc);
    }
    t.layer_piece.push_back((uint32_t)t.pieces.size());
    t.layers++;
  }
  t.total = total;
  t.stride = stride;
  return KAD_OK;
}

kad_status Engine::reduce(const Lane &L, const Tick &t, uint32_t begin, uint32_t count,
                          bool subtract) {
  HIP_TRY(launch_hit_reduce(t.out.path.p + (size_t)begin * t.stride, t.out.len.p + begin,
                            t.stride, count, tiles_hw_ * HIT_TILE_IDS, count_pool_.p, subtract,
                            subtract ? nullptr : group_pool_.p,
                            subtract ? nullptr : gmax_pool_.p, L.scratch(), L.rs));
  return KAD_OK;
}

kad_status Engine::launch(Lane &L, Tick &t) {
  hipStream_t s = L.s, rs = L.rs;
  const uint32_t np = (uint32_t)t.pieces.size();
  // fixed-size buffers, allocated on first use
  {
    kad_status st = t.out.ensure_entries(TICK_SAMPLES, TICK_PATH_BYTES / 4, rs);
    if (st) return st;
  }
  HIP_TRY(t.d_segs.ensure(MAX_PIECES));
  HIP_TRY(t.h_segs.ensure(MAX_PIECES));
  HIP_TRY(t.d_gat.ensure(MAX_PIECES));
  HIP_TRY(t.h_gat.ensure(MAX_PIECES));
  HIP_TRY(t.wlist.ensure(TICK_SAMPLES));
  HIP_TRY(t.wlist2.ensure(TICK_SAMPLES));
  if (L.bins.n == 0) {
    HIP_TRY(L.bins.ensure(TICK_PATH_BYTES / 4));
    L.bins_cap = TICK_PATH_BYTES / 4;
  }
  uint64_t max_layer = 0;
  for (uint32_t ly = 0; ly < t.layers; ++ly) {
    const Piece &a = t.pieces[t.layer_piece[ly]];
    const Piece &b = t.pieces[t.layer_piece[ly + 1] - 1];
    max_layer = std::max<uint64_t>(max_layer, b.begin + b.count - a.begin);
  }
  const uint64_t need_bins = max_layer * std::max<uint32_t>(t.stride - 2, 1);
  if (need_bins > L.bins_cap) return fail(KAD_EINVAL, "internal: hit bins too small");
  // segments
  for (uint32_t j = 0; j < np; ++j) {
    const Piece &pc = t.pieces[j];
    const kad_graph *g = pc.q->g;
    SampleSeg &sg = t.h_segs.p[j];
    sg.row = g->d_row;
    sg.col = g->d_col;
    sg.rrow = g->directed ? g->d_rrow : g->d_row;
    sg.rcol = g->directed ? g->d_rcol : g->d_col;
    sg.seed = pc.q->p.seed;
    sg.first = pc.first;
    sg.n = g->n;
    sg.phase = pc.kind == Kind::Pilot || pc.kind == Kind::PilotLast ? 0u : 1u;
    sg.begin = pc.begin;
    sg.id_base = (uint32_t)pc.q->base();
    sg.wide_only = pc.q->ovc == 2 ? 1u : 0u;
    sg.forward = g->search == KAD_SEARCH_FORWARD ? 1u : 0u;
  }
  // snapshots, layer by layer
  std::vector<GatherDesc> gat;
  t.layer_gat.assign(1, 0);
  t.layer_blocks.clear();
  t.layer_snap.assign(1, 0);
  uint64_t snap = 0;
  for (uint32_t ly = 0; ly < t.layers; ++ly) {
    uint32_t blocks = 0;
    for (uint32_t j = t.layer_piece[ly]; j < t.layer_piece[ly + 1]; ++j) {
      Piece &pc = t.pieces[j];
      GatherDesc d{};
      if (pc.kind == Kind::Pilot) continue;
      const Query *q = pc.q;
      d.off = q->base();
      d.dst = snap;
      if (pc.kind == Kind::PilotLast) {
        d.len = q->n;
        d.mode = GATHER_COUNT_ZERO;  // count0, and the counters restart for phase 1
      } else if (pc.kind == Kind::MainFull) {
        d.len = q->n;
        d.mode = GATHER_COUNT;
      } else {
        d.len = (uint32_t)q->checker->groups();
        d.mode = GATHER_GMAX;
      }
      d.block0 = blocks;
      blocks += (d.len + GATHER_CHUNK - 1) / GATHER_CHUNK;
      pc.snap = snap;
      snap += d.len;
      if (d.len) gat.push_back(d);
      else pc.snap = snap;  // empty snapshot
    }
    t.layer_gat.push_back((uint32_t)gat.size());
    t.layer_blocks.push_back(blocks);
    t.layer_snap.push_back(snap);
  }
  if (!gat.empty()) memcpy(t.h_gat.p, gat.data(), gat.size() * sizeof(GatherDesc));
  if (t.d_snap.n < snap) grow(t.d_snap, snap);
  if (t.h_snap.n < snap) grow(t.h_snap, snap);
  if (!t.d_snap.p || !t.h_snap.p) return fail(KAD_ENOMEM, "snapshot buffers");
  while (t.layer_ev.size() < t.layers) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    t.layer_ev.push_back(e);
  }
  // ---- sampler
  HIP_TRY(hipStreamWaitEvent(s, t.out.reduced, 0));
  static_assert(sizeof(SampleSeg) % 8 == 0 && sizeof(GatherDesc) % 8 == 0, "copied as words");
  // launch shape of the graph with the most samples in this launch
  const kad_graph *major = nullptr;
  {
    std::map<const kad_graph *, uint64_t> by_graph;
    uint64_t most = 0;
    for (const Piece &pc : t.pieces) {
      const uint64_t c = by_graph[pc.q->g] += pc.count;
      if (c > most) {
        most = c;
        major = pc.q->g;
      }
    }
  }
  const LaunchShape shape = graph_shape(major);
  const bool wide_lane = &L == &lanes_[1];
  if (L.nwslots == 0) return fail(KAD_ENOMEM, "no wide-count slots for this launch");
  int per_cu = 1;
  for (int j = 0; j < 3; ++j)
    if (SAMPLER_BLOCKS[j] == shape.block) per_cu = sampler_per_cu(ctx_, shape.block);
  // Lane 1's wide-count workgroups in flight each fill a CU for as long as their samples
  // take (hundreds of ms on a high-diameter graph); lane 0's sampler grid takes only the
  // CUs they leave, so that all its workgroups are resident at once: one that waited for
  // a CU would hold its sample ids, and so the tick, until the wide kernel finished.
  const uint32_t held =
      wide_lane ? 0u : (lanes_[1].wide_in_flight() + ctx_->wide_per_cu - 1) / ctx_->wide_per_cu;
  const bool shared = held > 0;
  const uint32_t free_cus = held < ctx_->cus ? ctx_->cus - held : 1u;
  const uint32_t resident = (uint32_t)std::min<uint64_t>(L.nslots, (uint64_t)free_cus * per_cu);
  // While lane 0 has work (and always in a server), the wide lane's launches take at most
  // a quarter of the CUs: a wide-count workgroup fills a CU's registers, and lane 1's long
  // high-diameter queries would otherwise hold most of the GPU away from every other query.
  WideState w1 = lane_wide(L);
  const bool capped = wide_lane && (lanes_[0].busy() || serving_);
  if (capped) w1.slots = std::min(w1.slots, std::max<uint32_t>(1, ctx_->cus / 4));
  const WideState w2 = lane_wide2(L);
  // The sampling chain: segment table to the device, counters cleared, the sampler (lane 0),
  // the wide-count passes (every sample of lane 1; in lane 0 the samples its sampler left:
  // counts past 128 bits, wide_only segments, more candidate edges than a slot holds; with
  // large arenas in two passes, the samples the lane's first pass cannot hold are sampled
  // again by fewer slots with larger arenas in the lane's same memory), the fix count to
  // the host.  With bd (a replay) the segment count, the sample count and the stride come
  // from the descriptor and the launches are sized for the largest tick.
  auto chain = [&](hipStream_t cs, const BatchDesc *bd) -> kad_status {
    const uint32_t nseg = bd ? MAX_PIECES : np, total = bd ? TICK_SAMPLES : t.total;
    const uint32_t stride = bd ? 0u : t.stride;
    if (bd)
      HIP_TRY(launch_copy_u64(reinterpret_cast<uint64_t *>(t.d_bd.p),
                              reinterpret_cast<const uint64_t *>(t.h_bd.p),
                              sizeof(BatchDesc) / 8, cs));
    HIP_TRY(launch_copy_u64((uint64_t *)t.d_segs.p, (const uint64_t *)t.h_segs.p,
                            (uint64_t)nseg * sizeof(SampleSeg) / 8, cs, bd,
                            sizeof(SampleSeg) / 8, true));
    HIP_TRY(launch_zero_u32(t.work.p, WORK_WORDS, cs));
    if (!bd && ctx_->timing) HIP_TRY(hipEventRecord(t.out.k0, cs));
    if (!wide_lane) {
      SampleOut so = t.out.view(stride);
      so.fix_list = t.wlist.p;
      so.fix_count = t.work.p + 1;
      HIP_TRY(launch_sampler_multi(t.d_segs.p, nseg, lane_slots(L, false), total, t.work.p, so,
                                   std::min(resident, total), shape, cs, bd));
    }
    SampleOut o1 = t.out.view(stride);
    if (w2.slots) {
      o1.fix_list = t.wlist2.p;
      o1.fix_count = t.work.p + 3;
    }
    HIP_TRY(launch_wide_fix(GraphDev{}, 0, 0, 0, t.d_segs.p, nseg, lane_slots(L, true),
                            w1, total, wide_lane, t.wlist.p, t.work.p + 1,
                            t.work.p + 2, o1, cs, bd));
    if (w2.slots)
      HIP_TRY(launch_wide_fix(GraphDev{}, 0, 0, 0, t.d_segs.p, nseg, lane_slots(L, true), w2,
                              total, false, t.wlist2.p, t.work.p + 3, t.work.p + 4,
                              t.out.view(stride), cs, bd));
    if (!wide_lane) HIP_TRY(launch_copy_u32(t.out.h_nwide.p, t.work.p + 1, 1, cs));
    if (bd) {  // the host mirrors, inside the chain
      HIP_TRY(launch_copy_u32(t.out.h_flags.p, t.out.flags.p, TICK_SAMPLES, cs, bd));
      HIP_TRY(launch_copy_u64(t.out.h_arcs.p, t.out.arcs.p, TICK_SAMPLES, cs, bd));
    }
    return KAD_OK;
  };
  const bool replay = ctx_->exec == KAD_EXEC_GRAPH && !ctx_->timing;
  if (replay) {
    HIP_TRY(t.h_bd.ensure(1));
    HIP_TRY(t.d_bd.ensure(1));
    // per block size, one chain for each lane-1 share (capped or not) and each lane-0 grid
    // (the whole GPU, or beside wide-count workgroups)
    BatchGraph &bg = t.chains[2 * (shape.block == 64 ? 0 : (shape.block == 128 ? 1 : 2)) +
                              (capped || shared ? 1 : 0)];
    ChainKey key;
    key << 3 << (int)(&L - lanes_) << shape.block << shape.small_exp << resident << wide_lane
        << lane_slots(L, false) << lane_slots(L, true) << w1 << w2
        << t.out.view(0) << t.out.h_flags.p << t.out.h_arcs.p << t.out.h_nwide.p << t.d_segs.p
        << t.h_segs.p << t.work.p << t.wlist.p << t.wlist2.p << t.h_bd.p << t.d_bd.p;
    kad_status st = record_chain(ctx_, bg, key,
                                 [&](hipStream_t cs) { return chain(cs, t.d_bd.p); });
    if (st) return st;
    // this tick's previous replay read its descriptor: the host has waited for its mirrors
    t.h_bd.p[0] = BatchDesc{0, 0, t.total, 0u, 0u, np, t.stride, 0u};
    HIP_TRY(hipGraphLaunch(bg.exec, s));
    bg.replays++;
    ctx_->chain_replays++;
  } else {
    kad_status st = chain(s, nullptr);
    if (st) return st;
  }
  if (wide_lane) t.out.h_nwide.p[0] = t.total;
  if (!replay && ctx_->timing) HIP_TRY(hipEventRecord(t.out.k1, s));
  HIP_TRY(hipEventRecord(t.sampled, s));
  // host copies by kernels: runtime copies were seen waiting for the other lane's kernels
  if (!replay) {
    HIP_TRY(launch_copy_u32(t.out.h_flags.p, t.out.flags.p, t.total, s));
    HIP_TRY(launch_copy_u64(t.out.h_arcs.p, t.out.arcs.p, t.total, s));
  }
  if (ctx_->timing) {
    HIP_TRY(launch_copy_u32(t.out.h_nodes.p, t.out.nodes.p, t.total, s));
    HIP_TRY(launch_copy_u32(t.out.h_len.p, t.out.len.p, t.total, s));
  }
  HIP_TRY(hipEventRecord(t.out.copied, s));
  // ---- per layer: hits into the pool, then the snapshot of each query's check
  HIP_TRY(hipStreamWaitEvent(rs, t.sampled, 0));
  if (!gat.empty())
    HIP_TRY(launch_copy_u64((uint64_t *)t.d_gat.p, (const uint64_t *)t.h_gat.p,
                            gat.size() * sizeof(GatherDesc) / 8, rs));
  for (uint32_t ly = 0; ly < t.layers; ++ly) {
    const Piece &a = t.pieces[t.layer_piece[ly]];
    const Piece &b = t.pieces[t.layer_piece[ly + 1] - 1];
    kad_status st = reduce(L, t, a.begin, b.begin + b.count - a.begin, false);
    if (st) return st;
    const uint32_t g0 = t.layer_gat[ly], g1 = t.layer_gat[ly + 1];
    if (g1 > g0) {
      HIP_TRY(launch_gather(t.d_gat.p + g0, g1 - g0, t.layer_blocks[ly], count_pool_.p,
                            gmax_pool_.p, t.d_snap.p, rs));
      const uint64_t s0 = t.layer_snap[ly], s1 = t.layer_snap[ly + 1];
      HIP_TRY(launch_copy_u64(t.h_snap.p + s0, t.d_snap.p + s0, s1 - s0, rs));
    }
    HIP_TRY(hipEventRecord(t.layer_ev[ly], rs));
  }
  t.wide_wgs = wide_lane ? w1.slots : 0u;
  t.in_flight = true;
  ticks_launched_++;
  samples_launched_ += t.total;
  return KAD_OK;
}

// A query stops after piece `at` of tick t: its hits from later pieces of t and from
// the tick in flight are subtracted, then its counters are read and reset.
kad_status Engine::stop_query(Query *q, Lane &L, Tick &t, size_t at, Tick &other) {
  hipStream_t rs = L.rs;
  if (q->status == KAD_OK) {
    for (size_t j = at + 1; j < t.pieces.size(); ++j)
      if (t.pieces[j].q == q) {
        kad_status st = reduce(L, t, t.pieces[j].begin, t.pieces[j].count, true);
        if (st) return st;
      }
    if (other.in_flight)
      for (const Piece &pc : other.pieces)
        if (pc.q == q) {
          kad_status st = reduce(L, other, pc.begin, pc.count, true);
          if (st) return st;
        }
    HIP_TRY(launch_copy_u64(final_pool_.p + q->base(), count_pool_.p + q->base(), q->n, rs));
  }
  HIP_TRY(launch_zero_u32((uint32_t *)(count_pool_.p + q->base()), 2ull * q->n, rs));
  HIP_TRY(hipEventRecord(q->final_ev, rs));
  q->st = QState::Final;
  q->t_final = clk::now();
  return KAD_OK;
}

kad_status Engine::process(Lane &L, Tick &t, Tick &other) {
  hipStream_t rs = L.rs;
  HIP_TRY(hipEventSynchronize(t.out.copied));
  if (ctx_->timing) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, t.out.k0, t.out.k1));
    ctx_->t_launches += 1;
    ctx_->t_samples += t.total;
    ctx_->t_seconds += ms * 1e-3;
    ctx_->t_wide += t.out.h_nwide.p[0];
    for (uint32_t k = 0; k < t.total; ++k) {
      ctx_->t_arcs += t.out.h_arcs.p[k];
      ctx_->t_nodes += t.out.h_nodes.p[k];
      ctx_->t_hits += t.out.h_len.p[k] >= 2 ? t.out.h_len.p[k] - 2 : 0;
    }
  }
  for (uint32_t ly = 0; ly < t.layers; ++ly) {
    HIP_TRY(hipEventSynchronize(t.layer_ev[ly]));
    for (uint32_t j = t.layer_piece[ly]; j < t.layer_piece[ly + 1]; ++j) {
      const Piece &pc = t.pieces[j];
      Query *q = pc.q;
      if (q->st == QState::Final || q->st == QState::Done) continue;  // past its stop
      uint64_t arcs = 0;
      uint32_t bad = 0;
      for (uint32_t k = pc.begin; k < pc.begin + pc.count; ++k) {
        arcs += t.out.h_arcs.p[k];
        bad |= t.out.h_flags.p[k];
      }
      if (bad) {
        if (bad & FLAG_OVERFLOW)
          finish_failed(q, KAD_EOVERFLOW, "a path count exceeded 128 bits");
        else if (bad & FLAG_RNG)
          finish_failed(q, KAD_ERNG, "bounded draw rejected 64 times");
        else
          finish_failed(q, KAD_EOVERFLOW, "candidate-edge list or path outgrew its buffer");
        kad_status st = stop_query(q, L, t, j, other);
        if (st) return st;
        continue;
      }
      if (pc.kind == Kind::Pilot || pc.kind == Kind::PilotLast) {
        q->pilot_arcs += arcs;
        if (pc.kind == Kind::Pilot) continue;
        // ---- computeDelta (Algorithm 2) on the pilot counts, beside the engine thread: on
        // a graph of millions of nodes it takes tens of ms, and every other query would wait
        const uint32_t n = q->n;
        q->count0.assign(t.h_snap.p + pc.snap, t.h_snap.p + pc.snap + n);
        q->t_pilot = clk::now();
        // the query's own range of the pinned group staging area, filled by the task
        uint32_t *stage = group_stage_.p + q->base();
        q->delta_task = std::async(std::launch::async, [q, n, stage] {
          q->lam_l.assign(n, q->p.epsilon);
          q->lam_u.assign(n, q->p.epsilon);
          q->L_l.resize(n);
          q->L_u.resize(n);
          if (q->p.mode == KAD_TOPK)
            topk_lambdas(n, q->p.k, q->count0.data(), q->alpha, q->p.epsilon, q->lam_l.data(),
                         q->lam_u.data());
          Groups groups;
          compute_delta(n, q->count0.data(), q->alpha, q->omega, q->lam_l.data(),
                        q->lam_u.data(), q->p.delta, q->eb, q->L_l.data(), q->L_u.data(), &q->C,
                        &groups);
          q->checker.reset(new StopChecker(n, q->p.mode, q->p.k, q->p.epsilon, q->omega,
                                           q->L_l.data(), q->L_u.data(), std::move(groups)));
          // group ids as pool ids, staged for the device copy
          const auto &go = q->checker->group_of();
          const uint32_t base = (uint32_t)q->base();
          parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned) {
            for (uint32_t v = vb; v < ve; ++v) stage[v] = go[v] + base;
          });
        });
        continue;
      }
      // ---- a main-phase check point (every B samples, or omega)
      q->arcs += arcs;
      q->tau += pc.count;
      bool stop = false;
      if (q->tau >= q->omega) {
        stop = true;
      } else if (pc.count == q->B) {
        const uint64_t *sp = t.h_snap.p + pc.snap;
        if (pc.kind == Kind::MainFull) {
          stop = q->checker->check(sp, q->tau);
        } else {
          stop = q->checker->check_group_max(sp, q->tau, &q->worst);
        }
        q->rule = stop;
      }
      if (stop) {
        kad_status st = stop_query(q, L, t, j, other);
        if (st) return st;
      }
    }
  }
  for (Query *q : t.queries) q->refs--;
  HIP_TRY(hipEventRecord(t.out.reduced, rs));
  t.in_flight = false;
  return KAD_OK;
}

kad_status Engine::cancel_all() {
  for (Query *q : active_) {
    if (q->st == QState::Final || q->st == QState::Done) continue;
    hipStream_t rs = lanes_[q->lane].rs;
    finish_failed(q, KAD_ECANCELED, "canceled");
    HIP_TRY(launch_zero_u32((uint32_t *)(count_pool_.p + q->base()), 2ull * q->n, rs));
    HIP_TRY(hipEventRecord(q->final_ev, rs));
    q->st = QState::Final;
    q->t_final = clk::now();
  }
  while (!queue_.empty()) {
    Query *q = queue_.front();
    queue_.pop_front();
    finish_failed(q, KAD_ECANCELED, "canceled before admission");
    q->st = QState::Done;
    q->t_admit = q->t_pilot = q->t_delta = q->t_final = q->t_done = clk::now();
    done_.push_back(q);
  }
  return KAD_OK;
}

kad_status Engine::finalize(bool block) {
  for (size_t j = 0; j < active_.size();) {
    Query *q = active_[j];
    if (q->st != QState::Final || q->refs > 0) {
      ++j;
      continue;
    }
    // a query canceled or failed while its computeDelta task ran: the task reads count0 and
    // writes the checker, which are released below
    if (q->delta_task.valid()) {
      if (!block && q->delta_task.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
        out_pending_ = true;
        ++j;
        continue;
      }
      q->delta_task.get();
    }
    if (q->out_task.valid()) {  // outputs under way: done once the task is
      if (!block && q->out_task.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
        out_pending_ = true;
        ++j;
        continue;
      }
      q->out_task.get();
      release_tiles(q);
      q->checker.reset();
      q->count0.clear();
      q->count0.shrink_to_fit();
      q->st = QState::Done;
      q->t_done = clk::now();
      done_.push_back(q);
      active_.erase(active_.begin() + j);
      continue;
    }
    if (block) {
      HIP_TRY(hipEventSynchronize(q->final_ev));
    } else {
      const hipError_t e = hipEventQuery(q->final_ev);
      if (e == hipErrorNotReady) {
        ++j;
        continue;
      }
      HIP_TRY(e);
    }
    if (q->status == KAD_OK) {
      const uint32_t n = q->n;
      kad_result *d = q->direct;
      auto pick64 = [n](uint64_t *caller, std::vector<uint64_t> &own) {
        return caller ? caller : (own.resize(n), own.data());
      };
      auto pickd = [n](double *caller, std::vector<double> &own) {
        return caller ? caller : (own.resize(n), own.data());
      };
      q->o_count = pick64(d ? d->count : nullptr, q->count);
      q->o_bc = pickd(d ? d->bc : nullptr, q->bc);
      q->o_lo = pickd(d ? d->lower : nullptr, q->lo);
      q->o_hi = pickd(d ? d->upper : nullptr, q->hi);
      // O(n) on graphs of millions of nodes: beside the engine thread (the query's counter
      // tiles, which the task reads, are released once it is done)
      const uint64_t *fin = final_pool_.p + q->base();
      q->out_task = std::async(std::launch::async, [q, n, fin] {
        memcpy(q->o_count, fin, (size_t)n * 8);
        node_outputs(n, q->o_count, q->tau, q->omega, q->rule, q->p.epsilon, q->L_l.data(),
                     q->L_u.data(), q->checker->group_of(), q->o_bc, q->o_lo, q->o_hi);
        if (q->p.mode == KAD_TOPK)
          topk_select(n, q->p.k, q->o_count, q->o_lo, q->o_hi, q->topk, q->rlo, q->rhi);
      });
      out_pending_ = true;
      ++j;
      continue;
    }
    release_tiles(q);
    q->checker.reset();
    q->count0.clear();
    q->count0.shrink_to_fit();
    q->st = QState::Done;
    q->t_done = clk::now();
    done_.push_back(q);
    active_.erase(active_.begin() + j);
  }
  return KAD_OK;
}

kad_status Engine::delta_done() {
  delta_pending_ = false;
  for (Query *q : active_) {
    if (!q->delta_task.valid() || q->status != KAD_OK || q->st != QState::Pilot) continue;
    if (q->delta_task.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
      delta_pending_ = true;
      continue;
    }
    q->delta_task.get();
    // group ids into the pool (staged by the task); the group maxima start at 0 with the
    // counters
    hipStream_t rs = lanes_[q->lane].rs;
    const uint32_t n = q->n, base = (uint32_t)q->base();
    HIP_TRY(launch_copy_u32(group_pool_.p + base, group_stage_.p + base, n, rs));
    HIP_TRY(launch_zero_u32((uint32_t *)(gmax_pool_.p + base), 2ull * q->checker->groups(), rs));
    q->delta_ready = true;
    q->st = QState::Main;
    q->t_delta = clk::now();
  }
  return KAD_OK;
}

kad_status Engine::step() {
  kad_status st = admit();
  if (st) return st;
  if ((st = delta_done())) return st;
  bool acted = false;
  for (int li = 0; li < 2; ++li) {
    Lane &L = lanes_[li];
    Tick &newer = L.ticks[L.cur], &older = L.ticks[1 - L.cur];
    if (!newer.in_flight) {
      if ((st = build(li, newer))) return st;
      if (newer.total > 0) {
        if ((st = launch(L, newer))) return st;
        acted = true;
      }
    }
    // lane 0's running tick is waited for; lane 1's only evaluated once complete
    if (older.in_flight) {
      if (li == 0 || tick_complete(older)) {
        if ((st = process(L, older, newer))) return st;
        L.cur = 1 - L.cur;
        acted = true;
      }
    } else if (newer.in_flight) {
      L.cur = 1 - L.cur;
    }
  }
  // block on a stopped query's counters only when nothing else can move
  const bool idle = !lanes_[0].busy() && !lanes_[1].busy();
  if (idle && (!grave_dev_.empty() || !grave_host_.empty())) release_graveyard();
  out_pending_ = false;
  st = finalize(idle);
  if (!acted && (!idle || delta_pending_ || out_pending_))
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  return st;
}

kad_status context_engine(kad_ctx *ctx, Engine **out) {
  if (!ctx->engine) {
    std::unique_ptr<Engine> e(new Engine(ctx));
    kad_status st = e->init();
    if (st) return st;
    ctx->engine = e.release();
  }
  *out = ctx->engine;
  return KAD_OK;
}

void destroy_engine(Engine *e) { delete e; }

// Let a query's host tasks end (computeDelta reads its pilot counts; the outputs task reads
// the engine's final-count pool), so that the engine may be destroyed.
void wait_tasks(Query *q) {
  if (q->delta_task.valid()) q->delta_task.wait();
  if (q->out_task.valid()) q->out_task.wait();
}

}  // namespace kad

// ---------------------------------------------------------------- C ABI

namespace {

void fill_result(const kad::Query *q, kad_result *r, kad_status *ret) {
  r->tau = q->tau;
  r->omega = q->omega;
  r->alpha = q->alpha;
  r->interval = q->B;
  r->arcs_scanned = q->arcs;
  r->pilot_arcs_scanned = q->pilot_arcs;
  r->overflow_samples = 0;  // not tracked per query by the engine
  r->vd = q->vd;
  r->vd_exact = q->vd_exact ? 1u : 0u;
  r->stop_reason = q->rule ? KAD_STOP_RULE : KAD_STOP_OMEGA;
  r->n = q->n;
  r->items = q->n;  // the engine runs node betweenness only
  r->C = q->C;
  r->seconds = kad::secs(q->t_submit, q->t_done);
  r->seconds_setup = kad::secs(q->t_submit, q->t_admit);
  r->seconds_pilot = q->delta_ready ? kad::secs(q->t_admit, q->t_pilot) : 0.0;
  r->seconds_delta = q->delta_ready ? kad::secs(q->t_pilot, q->t_delta) : 0.0;
  r->seconds_main = q->delta_ready ? kad::secs(q->t_delta, q->t_final) : 0.0;
  r->topk_len = 0;
  *ret = q->status;
  if (q->status != KAD_OK) return;
  const size_t n = q->n;
  if (r->count && r->count != q->o_count) memcpy(r->count, q->o_count, n * 8);
  if (r->bc && r->bc != q->o_bc) memcpy(r->bc, q->o_bc, n * 8);
  if (r->lower && r->lower != q->o_lo) memcpy(r->lower, q->o_lo, n * 8);
  if (r->upper && r->upper != q->o_hi) memcpy(r->upper, q->o_hi, n * 8);
  if (q->p.mode == KAD_TOPK) {
    r->topk_len = (uint32_t)q->topk.size();
    if (q->topk.size() > r->topk_cap) {
      *ret = kad::fail(KAD_ETOOSMALL, "top-k output needs %zu entries", q->topk.size());
      return;
    }
    for (size_t j = 0; j < q->topk.size(); ++j) {
      if (r->topk_node) r->topk_node[j] = q->topk[j];
      if (r->rank_lo) r->rank_lo[j] = q->rlo[j];
      if (r->rank_hi) r->rank_hi[j] = q->rhi[j];
    }
  }
}

}  // namespace

struct kad_server {
  kad_ctx *ctx = nullptr;
  kad::Engine *eng = nullptr;  // the context's engine
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<kad::Query *> incoming;
  std::map<uint64_t, std::unique_ptr<kad::Query>> queries;  // submitted, not yet retrieved
  std::map<uint64_t, bool> finished;
  uint64_t next_ticket = 1;
  bool quit = false;
  uint64_t cancel_req = 0, cancel_done = 0;  // kad_server_cancel calls, and those handled
  kad_status fatal = KAD_OK;
  std::string fatal_msg;
  uint64_t completed = 0;
  uint64_t launches0 = 0, samples0 = 0;  // engine totals when the server started
};

namespace {

static void server_rounds(kad_server *sv) {
  (void)hipSetDevice(sv->ctx->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        return sv->quit || !sv->incoming.empty() || sv->eng->busy() ||
               sv->cancel_req != sv->cancel_done;
      });
      if (sv->quit && !sv->eng->busy()) break;
      while (!sv->incoming.empty()) {
        sv->eng->enqueue(sv->incoming.front());
        sv->incoming.pop_front();
      }
    }
    kad_status st = KAD_OK;
    bool cancel = false;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      cancel = sv->cancel_req != sv->cancel_done;
      sv->cancel_done = sv->cancel_req;
    }
    try {
      if (cancel) st = sv->eng->cancel_all();
      if (!st && sv->eng->busy()) st = sv->eng->step();
    } catch (...) {
      st = kad::status_of_exception();
    }
    std::vector<kad::Query *> done = sv->eng->take_done();
    if (st || !done.empty()) {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (kad::Query *q : done) {
        sv->finished[q->ticket] = true;
        sv->completed++;
      }
      if (st) {
        sv->fatal = st;
        sv->fatal_msg = kad_last_error();
      }
      sv->cv_done.notify_all();
    }
    if (st) break;  // device error: every unfinished query reports it
  }
}

// The server's thread: rounds until destroyed.  A host failure outside the engine's steps
// (memory, in the server's own bookkeeping) stops it like a device error does: every
// unfinished query reports it, and no exception ends the process.
void server_loop(kad_server *sv) {
  try {
    server_rounds(sv);
  } catch (...) {
    const kad_status st = kad::status_of_exception();
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->fatal = st;
    sv->fatal_msg = kad_last_error();
    sv->cv_done.notify_all();
  }
}

kad_status server_take(kad_server *sv, uint64_t ticket, kad_result *r, std::unique_lock<std::mutex> &lk) {
  auto it = sv->queries.find(ticket);
  kad::Query *q = it->second.get();
  kad_status ret = KAD_OK;
  fill_result(q, r, &ret);
  if (ret != KAD_OK && q->status != KAD_OK) kad::fail(q->status, "%s", q->error.c_str());
  sv->finished.erase(ticket);
  std::unique_ptr<kad::Query> hold = std::move(it->second);
  sv->queries.erase(it);
  lk.unlock();
  hold.reset();
  return ret;
}

}  // namespace

extern "C" {

kad_status kad_run_batch(kad_ctx *ctx, uint32_t count, const kad_graph *const *graphs,
                         const kad_params *params, kad_result *results, kad_status *status) try {
  using kad::fail;
  if (!ctx || (count && (!graphs || !params || !results)))
    return fail(KAD_EINVAL, "NULL argument");
  for (uint32_t i = 0; i < count; ++i) {
    if (!graphs[i]) return fail(KAD_EINVAL, "graph %u is NULL", i);
    if (graphs[i]->ctx != ctx) return fail(KAD_EINVAL, "graph %u belongs to another context", i);
    kad_status st = kad::validate_params(graphs[i], &params[i]);
    if (st) return st;
    if (params[i].schedule != KAD_SCHEDULE_ADAPTIVE)
      return fail(KAD_EINVAL, "query %u: fixed schedules run through kad_run", i);
    if (params[i].target != KAD_TARGET_NODES)
      return fail(KAD_EINVAL, "query %u: edge betweenness runs through kad_run", i);
  }
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  kad::Engine *ep = nullptr;
  kad_status st = kad::context_engine(ctx, &ep);
  if (st) return st;
  kad::Engine &eng = *ep;
  std::vector<std::unique_ptr<kad::Query>> qs(count);
  const auto now = kad::clk::now();
  for (uint32_t i = 0; i < count; ++i) {
    qs[i].reset(new kad::Query());
    qs[i]->ticket = i;
    qs[i]->g = const_cast<kad_graph *>(graphs[i]);
    qs[i]->p = params[i];
    qs[i]->direct = &results[i];
    qs[i]->t_submit = now;
    eng.enqueue(qs[i].get());
  }
  // on a failure the engine may still point at this call's queries, and their host tasks
  // at its pools: those end first, and the next call starts with a new engine
  auto drop_engine = [&](kad_status why) {
    std::string msg = kad_last_error();
    for (auto &q : qs) kad::wait_tasks(q.get());
    kad::destroy_engine(ctx->engine);
    ctx->engine = nullptr;
    return fail(why, "%s", msg.c_str());
  };
  try {
    while (eng.busy())
      if ((st = eng.step())) return drop_engine(st);
  } catch (...) {
    return drop_engine(kad::status_of_exception());
  }
  (void)eng.take_done();  // every query of this call is done
  kad_status first = KAD_OK;
  std::string first_msg;
  for (uint32_t i = 0; i < count; ++i) {
    kad_status ri = KAD_OK;
    fill_result(qs[i].get(), &results[i], &ri);
    if (ri != KAD_OK && qs[i]->status != KAD_OK) kad::fail(ri, "%s", qs[i]->error.c_str());
    if (status) status[i] = ri;
    if (ri != KAD_OK && first == KAD_OK) {
      first = ri;
      first_msg = kad_last_error();
    }
  }
  if (first != KAD_OK) return fail(first, "%s", first_msg.c_str());
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_server_create(kad_ctx *ctx, kad_server **out) try {
  using kad::fail;
  if (!ctx || !out) return fail(KAD_EINVAL, "NULL argument");
  *out = nullptr;
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  std::unique_ptr<kad_server> sv(new kad_server());
  sv->ctx = ctx;
  kad_status st = kad::context_engine(ctx, &sv->eng);
  if (st) return st;
  sv->eng->set_serving(true);
  (void)sv->eng->take_done();
  sv->launches0 = sv->eng->ticks_launched();
  sv->samples0 = sv->eng->samples_launched();
  sv->th = std::thread(server_loop, sv.get());
  claim.release_to_owner();  // released by kad_server_destroy
  *out = sv.release();
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_server_submit(kad_server *sv, const kad_graph *g, const kad_params *p,
                             uint64_t *ticket) try {
  using kad::fail;
  if (!sv || !g || !p || !ticket) return fail(KAD_EINVAL, "NULL argument");
  if (g->ctx != sv->ctx) return fail(KAD_EINVAL, "the graph belongs to another context");
  kad_status st = kad::validate_params(g, p);
  if (st) return st;
  if (p->schedule != KAD_SCHEDULE_ADAPTIVE)
    return fail(KAD_EINVAL, "fixed schedules run through kad_run");
  if (p->target != KAD_TARGET_NODES) return fail(KAD_EINVAL, "edge betweenness runs through kad_run");
  std::unique_ptr<kad::Query> q(new kad::Query());
  q->g = const_cast<kad_graph *>(g);
  q->p = *p;
  q->t_submit = kad::clk::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->fatal) return fail(sv->fatal, "server stopped: %s", sv->fatal_msg.c_str());
  q->ticket = sv->next_ticket++;
  *ticket = q->ticket;
  sv->incoming.push_back(q.get());
  sv->queries[q->ticket] = std::move(q);
  sv->cv_work.notify_one();
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_server_poll(kad_server *sv, uint64_t ticket, kad_result *r) try {
  using kad::fail;
  if (!sv || !r) return fail(KAD_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (!sv->queries.count(ticket)) return fail(KAD_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (!sv->finished.count(ticket)) {
    if (sv->fatal) return fail(sv->fatal, "server stopped: %s", sv->fatal_msg.c_str());
    return fail(KAD_EBUSY, "query %llu is running", (unsigned long long)ticket);
  }
  return server_take(sv, ticket, r, lk);
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_server_wait(kad_server *sv, uint64_t ticket, kad_result *r, double timeout_s) try {
  using kad::fail;
  if (!sv || !r) return fail(KAD_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (!sv->queries.count(ticket)) return fail(KAD_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  auto ready = [&] {
    return sv->finished.count(ticket) > 0 || sv->fatal != KAD_OK || !sv->queries.count(ticket);
  };
  if (timeout_s < 0) {
    sv->cv_done.wait(lk, ready);
  } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return fail(KAD_EBUSY, "query %llu is still running", (unsigned long long)ticket);
  }
  if (!sv->queries.count(ticket))
    return fail(KAD_ECANCELED, "query %llu was dropped by kad_server_destroy", (unsigned long long)ticket);
  if (!sv->finished.count(ticket)) return fail(sv->fatal, "server stopped: %s", sv->fatal_msg.c_str());
  return server_take(sv, ticket, r, lk);
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_server_stats(kad_server *sv, uint64_t *completed, uint64_t *launches,
                            uint64_t *samples) try {
  if (!sv) return kad::fail(KAD_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (completed) *completed = sv->completed;
  if (launches) *launches = sv->eng->ticks_launched() - sv->launches0;
  if (samples) *samples = sv->eng->samples_launched() - sv->samples0;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_server_cancel(kad_server *sv) try {
  if (!sv) return kad::fail(KAD_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(sv->mu);
  for (kad::Query *q : sv->incoming) {  // not yet seen by the engine
    q->status = KAD_ECANCELED;
    q->error = "canceled before admission";
    q->t_admit = q->t_pilot = q->t_delta = q->t_final = q->t_done = kad::clk::now();
    sv->finished[q->ticket] = true;
  }
  sv->incoming.clear();
  sv->cancel_req++;
  sv->cv_work.notify_one();
  sv->cv_done.notify_all();
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_server_destroy(kad_server *sv) try {
  if (!sv) return KAD_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    // queries not yet admitted are dropped; admitted ones run to completion
    for (kad::Query *q : sv->incoming) sv->queries.erase(q->ticket);
    sv->incoming.clear();
    sv->quit = true;
    sv->cv_work.notify_one();
    sv->cv_done.notify_all();
  }
  if (sv->th.joinable()) sv->th.join();
  kad_ctx *ctx = sv->ctx;
  if (sv->eng) sv->eng->set_serving(false);
  if (sv->fatal) {  // the engine may still point at this server's queries
    for (auto &kv : sv->queries) kad::wait_tasks(kv.second.get());
    kad::destroy_engine(ctx->engine);
    ctx->engine = nullptr;
  }
  delete sv;
  ctx->busy.store(false);
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

}  // extern "C"
