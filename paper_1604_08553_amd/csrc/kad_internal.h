// Library-internal host structures shared by the single-run path (kad_runtime.cpp)
// and the multi-query engine (kad_engine.cpp).
#pragma once
#include <functional>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/kadabra.h"
#include "kad_device.h"

namespace kad {

kad_status fail(kad_status st, const char *fmt, ...);
// The status of the exception being handled, for the catch (...) handlers of the C entry
// points (no exception may cross the C boundary): host memory or threads exhausted give
// KAD_ENOMEM, anything else KAD_EINTERNAL, with the message set as fail() sets it.
kad_status status_of_exception();

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::kad::fail(KAD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t ensure(size_t count) {
    if (count <= n) return hipSuccess;
    release();
    hipError_t e = hipMalloc((void **)&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) n = count;
    return e;
  }
};

template <typename T>
struct PinBuf {
  T *p = nullptr;
  size_t n = 0;
  PinBuf() = default;
  PinBuf(const PinBuf &) = delete;
  PinBuf &operator=(const PinBuf &) = delete;
  ~PinBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t ensure(size_t count) {
    if (count <= n) return hipSuccess;
    release();
    // coherent: kernels may write it directly (see launch_to_host_*)
    hipError_t e = hipHostMalloc((void **)&p, std::max<size_t>(count, 1) * sizeof(T),
                                 hipHostMallocCoherent);
    if (e == hipSuccess) n = count;
    return e;
  }
};

constexpr uint32_t PI_CAP = 65536;  // candidate edges per slot (power of two)
constexpr uint32_t DEFAULT_BATCH = 65536;
// Counters of one sampler launch: [0] the sampler's sample counter, [1] its fix-list
// length, then the wide-count passes' ([2] the first pass's counter, [3] the length of
// its list for the second pass, [4] the second pass's counter).
constexpr uint32_t WORK_WORDS = 5;
// Wide-count arenas (limbs of 64 bits per slot) of graphs whose counts pass 128 bits: the
// first pass's size when a sample may need more (256 MiB), and the second pass's (1 GiB)
// unless the graph's worst case is smaller.
constexpr uint64_t WIDE_TIER1_LIMBS = 1ull << 25;
constexpr uint64_t WIDE_MAX_LIMBS = 1ull << 27;
// Sampler slot tables (kad_ctx_set_table): the sizes a caller may ask for, and the size the
// library takes when one record per node would leave fewer than TABLE_AUTO_PER_CU slots
// per CU.  A sample runs about 0.75x as fast with tables (probes, fewer resident
// workgroups), and below about four samples in flight per CU the dense layout loses more
// than that.  2^16 records hold the nodes one sample reaches before the two searches
// meet on the large power-law workloads (their largest sample over 10^5 draws reaches
// about 6K on a 10^6-node undirected graph, 21K on a 4*10^6-node directed one) with
// the table at most a third full.
constexpr uint32_t TABLE_MIN_BITS = 6, TABLE_MAX_BITS = 24, TABLE_AUTO_BITS = 16;
constexpr uint32_t TABLE_AUTO_PER_CU = 4;
// The wide-count kernel's own slots when the sampler's are tables: at most this share
// of the slot memory.
constexpr double WIDE_POOL_SHARE = 1.0 / 3.0;

// Device outputs of one sampler launch, with pinned host mirrors of the small ones.
struct OutSet {
  DevBuf<uint32_t> s, t, len, flags, nodes, path;
  DevBuf<uint32_t> fix_list;  // samples the sampler leaves to the wide-count kernel
  DevBuf<uint32_t> fix_list2; // samples the first wide pass leaves to the second
  DevBuf<uint32_t> epath, elen;  // edge betweenness: paths as edge ids (estride apart)
  uint32_t estride = 0;
  DevBuf<uint64_t> arcs;
  PinBuf<uint32_t> h_flags, h_len, h_nodes, h_nwide;  // h_nwide: samples resampled wide
  PinBuf<uint64_t> h_arcs;
  uint32_t cap = 0, stride = 0;
  hipEvent_t k0 = nullptr, k1 = nullptr;  // launch start/end (timing)
  hipEvent_t sampled = nullptr;           // sampler (and wide fix) done: paths final
  hipEvent_t copied = nullptr;            // sampler done and mirrors landed
  hipEvent_t reduced = nullptr;           // every reduction reading this set is done
  OutSet() = default;
  OutSet(const OutSet &) = delete;
  OutSet &operator=(const OutSet &) = delete;
  ~OutSet() {
    for (hipEvent_t e : {k0, k1, sampled, copied, reduced})
      if (e) (void)hipEventDestroy(e);
  }
  // capacity for `cap` samples of path stride `stride`; events created on first use
  // (`reduced` starts out recorded on `rs`)
  kad_status ensure(uint32_t cap, uint32_t stride, hipStream_t rs);
  // capacity for `cap` samples and `path_entries` path entries in all (any stride with
  // samples * stride <= path_entries)
  kad_status ensure_entries(uint32_t cap, uint64_t path_entries, hipStream_t rs);
  // fix_count: the launch's counter of fix_list entries (null: no list kept)
  SampleOut view(uint32_t path_stride, uint32_t *fix_count = nullptr) const;
  // room for `cap` samples' edge paths, `estride` entries apart
  kad_status ensure_edges(uint32_t cap, uint32_t estride);
};

// A chain of launches recorded once into a hipGraph and replayed; `key` lists everything
// the recording bakes in (buffer addresses, sizes, launch shapes), and a replay with
// another key records the chain again.
struct BatchGraph {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t records = 0, replays = 0;
  BatchGraph() = default;
  BatchGraph(const BatchGraph &) = delete;
  BatchGraph &operator=(const BatchGraph &) = delete;
  ~BatchGraph() { release(); }
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
};

// What a recorded chain bakes in, as words (addresses, sizes, launch shapes).
struct ChainKey {
  std::vector<uint64_t> v;
  template <typename T>
  ChainKey &operator<<(T x) {
    if constexpr (std::is_pointer<T>::value) v.push_back((uint64_t)(uintptr_t)x);
    else v.push_back((uint64_t)x);
    return *this;
  }
  ChainKey &operator<<(const GraphDev &g) {
    return *this << g.n << g.arcs << g.row << g.col << g.rrow << g.rcol << g.forward;
  }
  ChainKey &operator<<(const SlotState &t) {
    return *this << t.slots << t.n << t.pi_cap << t.rec << t.visit << t.pi << t.hbits << t.vh;
  }
  ChainKey &operator<<(const WideState &w) {
    return *this << w.slots << w.max_lev << w.arena_limbs << w.arena << w.lv << w.lbase;
  }
  ChainKey &operator<<(const SampleOut &o) {
    return *this << o.s << o.t << o.len << o.flags << o.nodes << o.arcs << o.path << o.stride
                 << o.fix_list << o.fix_count;
  }
};

class Engine;
void destroy_engine(Engine *e);

}  // namespace kad

struct kad_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // sampling (unless the caller gives one)
  hipStream_t pstream = nullptr;  // a run's first main batch, beside its pilot
  hipStream_t rstream = nullptr;  // hit reductions and check snapshots
  uint64_t budget = 0;
  uint64_t used_graphs = 0;
  uint32_t cus = 0;
  int blocks_per_cu[3] = {1, 1, 1};  // resident sampler workgroups per CU, per SAMPLER_BLOCKS
  int blocks_per_cu_tab[3] = {1, 1, 1};  // the same with slot tables
  int wide_per_cu = 1;               // resident wide-count workgroups per CU
  std::atomic<bool> busy{false};  // one user at a time (a call, or a server's engine)
  // per-slot working state.  slot_hbits = 0: every slot holds one record per node of the
  // largest graph seen (slot_n), and the wide-count kernel uses the first sampler slots.
  // slot_hbits > 0: sampler slots hold tables of 2^slot_hbits records whatever the graph
  // (SlotState::hbits); the wide-count kernel then has wpool slots of its own with one
  // record per node (slot_n = their node capacity).
  uint32_t slot_n = 0, slots = 0;
  uint64_t slot_bytes = 0;
  kad::DevBuf<uint32_t> rec, visit;  // node records (REC_WORDS words each), reached lists
  kad::DevBuf<uint64_t> pi;
  uint32_t slot_hbits = 0;
  uint32_t table_knob = 0;  // kad_ctx_set_table: 0 the library's choice, 1 dense, else log2 size
  kad::DevBuf<uint32_t> vh;  // tables: the record index of each reached-list entry
  uint32_t wpool = 0;
  kad::DevBuf<uint32_t> wrec, wvisit;
  kad::DevBuf<uint64_t> wpi;
  // wide-count resampling (kad::WideState): samples whose counts pass 128 bits or whose
  // candidate edges outgrow a slot.  w_big: the arena sized for wide counts (graphs whose
  // counts can pass 128 bits), else for the candidate edges of 128-bit graphs only.
  // Large arenas come in two passes over the same memory: w_slots slots of w_arena_limbs,
  // then, for the samples that outgrow those, w_slots2 slots of w_arena_limbs2 (0: none).
  uint32_t w_slots = 0, w_max_lev = 0, w_slots2 = 0;
  bool w_big = false;
  uint64_t run_wide = 0;  // samples resampled wide during the current kad_run
  uint64_t w_arena_limbs = 0, w_arena_limbs2 = 0;
  uint32_t w_user_slots = 0;  // kad_ctx_set_wide (0: the library's choice)
  uint64_t w_user_limbs = 0;
  kad::DevBuf<uint64_t> w_arena, w_lbase;
  kad::DevBuf<uint32_t> w_lv;
  // per-launch outputs, double-buffered so the next batch can be sampled while the
  // host checks the current one
  kad::OutSet outs[2];
  // counters of a launch (WORK_WORDS); work2: the same for pstream launches
  kad::DevBuf<uint32_t> work, work2, group;
  kad::DevBuf<uint64_t> count, gmax;
  hipEvent_t ev_s = nullptr, ev_rs = nullptr, ev_ps = nullptr;  // wait_stream's markers
  kad::DevBuf<uint64_t> count0d;         // pilot counts (all-nodes runs)
  kad::DevBuf<uint32_t> hist, cgrp;      // their histogram; count -> stopping group
  kad::PinBuf<uint32_t> h_hist, h_cgrp;
  kad::PinBuf<uint64_t> h_count0p;
  kad::DevBuf<uint32_t> bins, bin_count;  // hit-reduction scratch (bin_count all zero between calls)
  kad::DevBuf<uint32_t> tile_start, tile_fill;  // compact layout (tile_fill all zero between calls)
  uint64_t bins_cap = 0;
  bool bins_compact = false;
  kad::PinBuf<uint32_t> h_s, h_t, h_path;
  kad::PinBuf<uint64_t> h_count;
  kad::DevBuf<uint32_t> ivtmp;   // launch_hit_batch: hits per node and check interval
  kad::DevBuf<uint64_t> ivmax;   // launch_hit_batch: group maxima per check interval
  std::vector<hipEvent_t> chunk_ev;
  // host scratch of kad_run, kept across calls (large fresh allocations fault in pages)
  std::vector<uint64_t> h_count0;
  std::vector<double> h_lam_l, h_lam_u, h_L_l, h_L_u, h_bc, h_lo, h_hi;
  // timing of the sampler launches (HIP events on the launch stream)
  bool timing = false;
  uint64_t t_launches = 0, t_samples = 0, t_arcs = 0, t_nodes = 0, t_hits = 0, t_wide = 0;
  double t_seconds = 0.0;
  hipEvent_t t_ref = nullptr;                      // a run's timing reference
  bool t_run_ref = false;                          // t_ref holds the running kad_run's
  std::vector<std::pair<float, float>> t_iv;       // its launches' intervals (ms from t_ref)
  // the multi-query engine (kad_run_batch, kad_server_*), created on first use
  kad::Engine *engine = nullptr;
  // device address of the fixed scratch array used by kad_hit_counts_noalloc
  void *noalloc = nullptr;
  // how kad_run launches (KAD_EXEC_*); with KAD_EXEC_GRAPH its main-phase batches replay
  // recorded chains: per output set the sampling chain (bgraph[set]) and the batched
  // reduction (bgraph[2 + set]), reading the batch from d_bd[set] (copied from h_bd[set]
  // by the sampling chain).  cstream: the stream chains are recorded on.
  uint32_t exec = KAD_EXEC_GRAPH;
  hipStream_t cstream = nullptr;
  kad::BatchGraph bgraph[4];
  kad::PinBuf<kad::BatchDesc> h_bd;
  kad::DevBuf<kad::BatchDesc> d_bd;
  kad::PinBuf<uint64_t> snaps;  // kad_run's check snapshots, one per check of a batch
  // chains recorded and replayed, by kad_run and by the engine's ticks
  std::atomic<uint64_t> chain_records{0}, chain_replays{0};
  ~kad_ctx() {
    kad::destroy_engine(engine);
    for (auto e : chunk_ev) (void)hipEventDestroy(e);
  }
};

struct kad_graph {
  kad_ctx *ctx = nullptr;
  uint32_t n = 0;
  uint64_t arcs = 0;
  bool directed = false;
  std::vector<uint32_t> row, col, rrow, rcol;  // host copies
  uint32_t *d_row = nullptr, *d_col = nullptr, *d_rrow = nullptr, *d_rcol = nullptr;
  bool owns_fwd = false, owns_rev = false;
  uint64_t bytes = 0;
  std::mutex vd_mu;
  uint32_t vd = 0;
  bool vd_exact = false, vd_known = false;
  uint32_t maxdeg = 0;  // largest out- or in-degree
  kad::LaunchShape shape;  // sampler launch shape (kad_graph_set_launch / kad_autotune)
  bool shape_set = false;
  uint32_t search = 0;     // KAD_SEARCH_BALANCED or KAD_SEARCH_FORWARD
  // edge ids of an undirected graph's arcs (built on first use; directed graphs use the
  // arc position itself)
  std::mutex eid_mu;
  bool eid_ready = false;
  std::vector<uint32_t> eid;
  uint32_t *d_eid = nullptr;
};

namespace kad {

// Claims the context for the lifetime of the guard; ok() is false when it is in use.
class CtxClaim {
 public:
  explicit CtxClaim(kad_ctx *c) : c_(c) {
    bool expect = false;
    ok_ = c_->busy.compare_exchange_strong(expect, true);
  }
  ~CtxClaim() {
    if (ok_) c_->busy.store(false);
  }
  bool ok() const { return ok_; }
  void release_to_owner() { ok_ = false; }  // keep the claim past this guard

 private:
  kad_ctx *c_;
  bool ok_ = false;
};

// Record the launches `fn` makes on the stream it is given (the context's capture stream)
// into bg as a hipGraph, unless bg already holds a recording with this key.
kad_status record_chain(kad_ctx *ctx, BatchGraph &bg, const ChainKey &key,
                        const std::function<kad_status(hipStream_t)> &fn);

// The context's multi-query engine (created, with its counter pools, on first use).
kad_status context_engine(kad_ctx *ctx, Engine **out);

// Parameter checks shared by every entry point that runs Algorithm 1.
kad_status validate_params(const kad_graph *g, const kad_params *p);
// Items of a run: the nodes, or the edges (arcs, or arcs / 2 when undirected).
uint64_t run_items(const kad_graph *g, uint32_t target);
// The graph's edge-id map on the device (nullptr for a directed graph: the arc position
// is the id), built on first use.
kad_status graph_edge_ids(kad_graph *g, const uint32_t **d_eid);

GraphDev dev_view(const kad_graph *g);
// The graph's vertex diameter by the library rule, computed once (thread-safe).
kad_status graph_vd(kad_graph *g, uint32_t *vd, bool *exact);
// Slot state for graphs of up to n nodes (reallocates, and synchronises, when it grows).
kad_status ensure_slots(kad_ctx *ctx, uint32_t n);
SlotState slot_view(const kad_ctx *ctx, uint32_t slot0 = 0);
// The dense slots the wide-count kernel runs on: the sampler slots, or with slot tables
// the wide-count pool.
SlotState wide_slot_view(const kad_ctx *ctx, uint32_t slot0 = 0);
uint32_t wide_slot_count(const kad_ctx *ctx);
// Resident sampler workgroups per CU of this workgroup size in the context's slot layout.
int sampler_per_cu(const kad_ctx *ctx, int block);
WideState wide_view(const kad_ctx *ctx);
// The second wide pass's view of the same arena (slots 0 when there is none).
WideState wide_view2(const kad_ctx *ctx);
// Wide path counts: 0 = a graph whose path counts always fit 128 bits (VD and the
// largest degree bound them), 1 = overflowed samples are resampled wide, 2 = a
// high-diameter graph whose samples all go to the wide kernel.  vd_from_library:
// false for a caller's VD override, whose bound is not trusted (then 1).
int overflow_class(const kad_graph *g, uint32_t vd, bool vd_from_library);
// Wide working memory able to sample graph g (of overflow class ovc) again: every graph
// needs it, for samples with more candidate edges than a slot holds; a graph whose counts
// can pass 128 bits needs the large arena.  Allocated on first use, grown (after a device
// synchronisation) when a graph needs more.
kad_status ensure_wide(kad_ctx *ctx, const kad_graph *g, int ovc);
bool wide_fits(const kad_ctx *ctx, const kad_graph *g, int ovc);
// Launch the wide-count resampling of a launch of `count` samples whose outputs are
// `out`: the samples of its fix list (list, *list_count), or with `all` every sample (no
// sampler launch before); work: 3 counters, zero at launch.  With large arenas in two
// passes, list2 (room for count entries) carries the samples the first pass leaves to the
// second.  segs == nullptr: single graph g.  bd: as in launch_wide_fix.  slot0: the first
// sampler slot it may use (one record per node); with slot tables the passes take the
// wide-count pool from its first slot.
kad_status launch_wide(kad_ctx *ctx, const GraphDev &g, uint64_t seed, uint32_t phase,
                       uint64_t first, const SampleSeg *segs, uint32_t nseg, uint32_t count,
                       bool all, const uint32_t *list, const uint32_t *list_count,
                       uint32_t *work, uint32_t *list2, const SampleOut &out,
                       hipStream_t stream, uint32_t slot0 = 0, const BatchDesc *bd = nullptr);
// The graph's launch shape (set or tuned, else a default by size), and the grid of a
// launch of `count` samples with it.
LaunchShape graph_shape(const kad_graph *g);
uint32_t launch_grid(const kad_ctx *ctx, const LaunchShape &shape, uint64_t count,
                     uint32_t slot0 = 0);

// Per-node outputs of a finished run (Theorem 1 intervals and the top-k ranking).
// bc, lo, hi: length n.  With rule_stop the interval is [bc - f, bc + g], else
// [bc - eps, bc + eps].  group_of (may be empty) maps nodes to classes of identical
// (L_l, L_u), used to memoise f and g.
void node_outputs(uint32_t n, const uint64_t *cnt, uint64_t tau, uint64_t omega, bool rule_stop,
                  double eps, const double *L_l, const double *L_u,
                  const std::vector<uint32_t> &group_of, double *bc, double *lo, double *hi);
// The same outputs when node v's group is cgrp[count0[v]] (group L values gL_l, gL_u).
void node_outputs_pilot(uint32_t n, const uint64_t *cnt, uint64_t tau, uint64_t omega, bool rule,
                        double eps, const uint64_t *count0, const std::vector<uint32_t> &cgrp,
                        const std::vector<double> &gL_l, const std::vector<double> &gL_u,
                        double *bc, double *lo, double *hi, uint64_t *count_out,
                        const std::function<void(uint32_t)> &wait_to = nullptr);
// Top-k selection: nodes with rank_lo <= k ordered by (count desc, id asc).
void topk_select(uint32_t n, uint32_t k, const uint64_t *cnt, const double *lo, const double *hi,
                 std::vector<uint32_t> &sel, std::vector<uint32_t> &rlo_sel,
                 std::vector<uint32_t> &rhi_sel);

}  // namespace kad
