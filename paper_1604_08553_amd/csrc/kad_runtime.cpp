// C ABI of the sampled-betweenness library: contexts, graphs, the adaptive run
// (Algorithm 1 of Borassi & Natale with a batched stopping check) and the sampling
// primitives.  The sampling itself runs in the HIP kernels of kad_kernels.hip; this
// file moves data, schedules launches and evaluates the binary64 statistics.
#include <functional>
#include <atomic>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <memory>
#include <string>
#include <system_error>
#include <type_traits>
#include <vector>

#include "kad_internal.h"
#include "kad_stats.h"

namespace kad {

thread_local std::string g_error;

kad_status fail(kad_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

kad_status status_of_exception() {
  try {
    throw;
  } catch (const std::bad_alloc &) {
    return fail(KAD_ENOMEM, "host memory exhausted");
  } catch (const std::system_error &e) {
    return fail(KAD_ENOMEM, "host resources exhausted: %s", e.what());
  } catch (const std::exception &e) {
    return fail(KAD_EINTERNAL, "internal error: %s", e.what());
  } catch (...) {
    return fail(KAD_EINTERNAL, "internal error");
  }
}

kad_status OutSet::ensure(uint32_t want_cap, uint32_t want_stride, hipStream_t rs) {
  if (cap < want_cap || stride < want_stride) {
    const uint32_t c = std::max(want_cap, cap);
    const uint32_t st = std::max(want_stride, stride);
    for (auto *b : {&s, &t, &len, &flags, &nodes, &path, &fix_list, &fix_list2}) b->release();
    arcs.release();
    HIP_TRY(s.ensure(c));
    HIP_TRY(t.ensure(c));
    HIP_TRY(len.ensure(c));
    HIP_TRY(flags.ensure(c));
    HIP_TRY(nodes.ensure(c));
    HIP_TRY(fix_list.ensure(c));
    HIP_TRY(fix_list2.ensure(c));
    HIP_TRY(arcs.ensure(c));
    HIP_TRY(path.ensure((size_t)c * st));
    HIP_TRY(h_flags.ensure(c));
    HIP_TRY(h_nwide.ensure(1));
    HIP_TRY(h_len.ensure(c));
    HIP_TRY(h_nodes.ensure(c));
    HIP_TRY(h_arcs.ensure(c));
    cap = c;
    stride = st;
  }
  if (!k0) HIP_TRY(hipEventCreate(&k0));
  if (!k1) HIP_TRY(hipEventCreate(&k1));
  if (!sampled) HIP_TRY(hipEventCreateWithFlags(&sampled, hipEventDisableTiming));
  if (!copied) HIP_TRY(hipEventCreateWithFlags(&copied, hipEventDisableTiming));
  if (!reduced) {
    HIP_TRY(hipEventCreateWithFlags(&reduced, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(reduced, rs));  // nothing pending yet
  }
  return KAD_OK;
}

kad_status OutSet::ensure_entries(uint32_t want_cap, uint64_t path_entries, hipStream_t rs) {
  if (cap < want_cap || path.n < path_entries) {
    for (auto *b : {&s, &t, &len, &flags, &nodes, &path, &fix_list, &fix_list2}) b->release();
    arcs.release();
    HIP_TRY(s.ensure(want_cap));
    HIP_TRY(t.ensure(want_cap));
    HIP_TRY(len.ensure(want_cap));
    HIP_TRY(flags.ensure(want_cap));
    HIP_TRY(nodes.ensure(want_cap));
    HIP_TRY(fix_list.ensure(want_cap));
    HIP_TRY(fix_list2.ensure(want_cap));
    HIP_TRY(arcs.ensure(want_cap));
    HIP_TRY(path.ensure(path_entries));
    HIP_TRY(h_flags.ensure(want_cap));
    HIP_TRY(h_nwide.ensure(1));
    HIP_TRY(h_len.ensure(want_cap));
    HIP_TRY(h_nodes.ensure(want_cap));
    HIP_TRY(h_arcs.ensure(want_cap));
    cap = want_cap;
    stride = (uint32_t)std::min<uint64_t>(path_entries / std::max(want_cap, 1u), 0xFFFFFFFFu);
  }
  return ensure(cap, 0, rs);  // events
}

kad_status OutSet::ensure_edges(uint32_t want_cap, uint32_t want_estride) {
  if (epath.n < (size_t)want_cap * want_estride || elen.n < want_cap) {
    epath.release();
    elen.release();
    HIP_TRY(epath.ensure((size_t)want_cap * want_estride));
    HIP_TRY(elen.ensure(want_cap));
  }
  estride = want_estride;
  return KAD_OK;
}

SampleOut OutSet::view(uint32_t path_stride, uint32_t *fix_count) const {
  SampleOut so;
  so.s = s.p;
  so.t = t.p;
  so.len = len.p;
  so.flags = flags.p;
  so.nodes = nodes.p;
  so.arcs = arcs.p;
  so.path = path.p;
  so.stride = path_stride;
  so.fix_list = fix_count ? fix_list.p : nullptr;
  so.fix_count = fix_count;
  return so;
}

GraphDev dev_view(const kad_graph *g) {
  GraphDev d;
  d.n = g->n;
  d.arcs = g->arcs;
  d.row = g->d_row;
  d.col = g->d_col;
  d.rrow = g->directed ? g->d_rrow : g->d_row;
  d.rcol = g->directed ? g->d_rcol : g->d_col;
  d.forward = g->search == KAD_SEARCH_FORWARD ? 1u : 0u;
  return d;
}

kad_status graph_vd(kad_graph *g, uint32_t *vd, bool *exact) {
  std::lock_guard<std::mutex> lk(g->vd_mu);
  if (!g->vd_known) {
    bool ex = false;
    const uint32_t *rr = g->directed ? g->rrow.data() : g->row.data();
    const uint32_t *rc = g->directed ? g->rcol.data() : g->col.data();
    if (vertex_diameter(g->n, g->arcs, g->row.data(), g->col.data(), rr, rc, 1e9, &g->vd, &ex))
      return fail(KAD_EINVAL, "vertex diameter: bad graph");
    g->vd_exact = ex;
    g->vd_known = true;
  }
  *vd = g->vd;
  *exact = g->vd_exact;
  return KAD_OK;
}

kad_status ensure_slots(kad_ctx *ctx, uint32_t n) {
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->slot_n >= n && ctx->slots > 0) return KAD_OK;
  HIP_TRY(hipDeviceSynchronize());  // no launch may still use the old state
  ctx->rec.release();
  ctx->visit.release();
  ctx->vh.release();
  ctx->pi.release();
  ctx->wrec.release();
  ctx->wvisit.release();
  ctx->wpi.release();
  ctx->slots = ctx->wpool = 0;
  ctx->slot_n = 0;
  ctx->slot_hbits = 0;
  // the wide-count arena is laid out after the slots, from what they leave
  ctx->w_arena.release();
  ctx->w_lv.release();
  ctx->w_lbase.release();
  ctx->w_slots = ctx->w_slots2 = 0;
  ctx->w_arena_limbs = ctx->w_arena_limbs2 = 0;
  const uint32_t want_slots =
      ctx->cus * (uint32_t)*std::max_element(ctx->blocks_per_cu, ctx->blocks_per_cu + 3);
  const uint32_t want_tab =
      ctx->cus * (uint32_t)*std::max_element(ctx->blocks_per_cu_tab, ctx->blocks_per_cu_tab + 3);
  const uint64_t dense_slot = (uint64_t)n * (4ull * REC_WORDS + 4) + (uint64_t)PI_CAP * 8;
  // slots take at most 70% of what the budget leaves after the graphs and 1 GiB (the
  // wide-count arenas, the engine's pools and the run buffers use the rest)
  const uint64_t avail = ctx->budget > ctx->used_graphs + (1024ull << 20)
                             ? (uint64_t)(0.7 * (double)(ctx->budget - ctx->used_graphs - (1024ull << 20)))
                             : 0;
  // one record per node, unless that leaves fewer than TABLE_AUTO_PER_CU slots per CU (and
  // the graph is larger than a table) or the caller chose tables
  uint32_t hbits = 0;
  if (ctx->table_knob >= TABLE_MIN_BITS)
    hbits = ctx->table_knob;
  else if (ctx->table_knob == 0 && avail / dense_slot < (uint64_t)TABLE_AUTO_PER_CU * ctx->cus &&
           n > (1u << TABLE_AUTO_BITS))
    hbits = TABLE_AUTO_BITS;
  uint64_t slots = 0, wpool = 0, table_slot = 0;
  if (hbits == 0) {
    slots = std::min<uint64_t>(want_slots, avail / dense_slot);
  } else {
    // the wide-count kernel's dense slots first (as many as it can run resident, within
    // their share), then the tables: records, reached list, record indices, candidates
    const uint64_t H = 1ull << hbits;
    table_slot = H * (4ull * REC_WORDS + 8) + (uint64_t)PI_CAP * 8;
    wpool = std::min<uint64_t>(std::max<uint32_t>(16, (uint32_t)ctx->wide_per_cu * ctx->cus),
                               (uint64_t)(WIDE_POOL_SHARE * (double)avail) / dense_slot);
    slots = wpool ? std::min<uint64_t>(want_tab, (avail - wpool * dense_slot) / table_slot) : 0;
  }
  if (slots == 0)
    return fail(KAD_ENOMEM, "HBM budget too small for one sampler slot of a %u-node graph", n);
  const uint64_t cap = hbits ? (1ull << hbits) : n;  // records per sampler slot
  HIP_TRY(ctx->rec.ensure((size_t)(slots * cap * REC_WORDS)));
  HIP_TRY(ctx->visit.ensure((size_t)(slots * cap)));
  HIP_TRY(ctx->pi.ensure((size_t)slots * PI_CAP));
  HIP_TRY(hipMemsetAsync(ctx->rec.p, 0, (size_t)(slots * cap * 4 * REC_WORDS), ctx->stream));
  if (hbits) {
    HIP_TRY(ctx->vh.ensure((size_t)(slots * cap)));
    HIP_TRY(ctx->wrec.ensure((size_t)(wpool * n * REC_WORDS)));
    HIP_TRY(ctx->wvisit.ensure((size_t)(wpool * n)));
    HIP_TRY(ctx->wpi.ensure((size_t)(wpool * PI_CAP)));
    HIP_TRY(hipMemsetAsync(ctx->wrec.p, 0, (size_t)(wpool * n * 4 * REC_WORDS), ctx->stream));
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->slots = (uint32_t)slots;
  ctx->slot_n = n;
  ctx->slot_hbits = hbits;
  ctx->wpool = (uint32_t)wpool;
  ctx->slot_bytes = hbits ? slots * table_slot + wpool * dense_slot : slots * dense_slot;
  return KAD_OK;
}

// Limbs of one wide slot's arena for graph g: with counts that may pass 128 bits, at
// least 2^20; otherwise the counts of every node at three limbs, every arc as a candidate
// edge, and the selection's scratch.
static uint64_t wide_limbs_needed(const kad_graph *g, int ovc) {
  if (ovc != 0) return 1ull << 20;
  return std::min<uint64_t>(1ull << 27, 3ull * g->n + g->arcs + (1ull << 18));
}

// An arena that holds any sample of g: every node's count at the widest count's limbs
// (a count is below maxdeg^(VD-1)) plus two, every arc as a candidate edge with the
// product of two counts, and the selection's scratch (capped at 2^40).
static uint64_t wide_limbs_worst(const kad_graph *g) {
  const double vd = g->vd_known ? (double)g->vd : (double)g->n;
  const double bits = std::max(vd - 1.0, 1.0) * std::log2(std::max<double>(g->maxdeg, 2.0));
  const double L = std::ceil(bits / 64.0);
  const double w = (double)g->n * (L + 2.0) + (double)g->arcs * (2.0 * L + 2.0) + 262144.0;
  return (uint64_t)std::min(w, 1099511627776.0);
}

bool wide_fits(const kad_ctx *ctx, const kad_graph *g, int ovc) {
  if (ctx->w_slots == 0) return false;
  if (ovc == 0) return ctx->w_arena_limbs >= wide_limbs_needed(g, 0);
  if (!ctx->w_big) return false;
  if (ctx->w_user_limbs) return true;  // the caller's layout (kad_ctx_set_wide)
  const uint64_t worst = wide_limbs_worst(g);
  return ctx->w_arena_limbs >= worst ||
         (ctx->w_slots2 > 0 && ctx->w_arena_limbs2 >= std::min(worst, WIDE_MAX_LIMBS));
}

kad_status ensure_wide(kad_ctx *ctx, const kad_graph *g, int ovc) {
  if (wide_fits(ctx, g, ovc)) return KAD_OK;
  const bool big = ovc != 0 || ctx->w_big;
  const uint64_t want = std::max(wide_limbs_needed(g, ovc),
                                 ctx->w_slots ? ctx->w_arena_limbs : (uint64_t)0);
  HIP_TRY(hipDeviceSynchronize());  // no launch may still use the old arena
  ctx->w_arena.release();
  ctx->w_lv.release();
  ctx->w_lbase.release();
  ctx->w_slots = ctx->w_slots2 = 0;
  ctx->w_arena_limbs = ctx->w_arena_limbs2 = 0;
  const uint64_t left = ctx->budget > ctx->used_graphs + ctx->slot_bytes + (1024ull << 20)
                            ? ctx->budget - ctx->used_graphs - ctx->slot_bytes - (1024ull << 20)
                            : 0;
  const uint32_t max_lev = 16384;
  const uint64_t tables = 2ull * max_lev * (16 + 8);  // one slot's level tables
  uint32_t w_slots = 0, w_slots2 = 0;
  uint64_t limbs = 0, limbs2 = 0;
  if (!big) {
    // 128-bit graphs (candidate edges past a slot only): 16 slots, each with room for every
    // node's count at three limbs and every arc as a candidate edge
    w_slots = std::min<uint32_t>(16, wide_slot_count(ctx));
    limbs = want;
    if (w_slots == 0 || left / 2 < (uint64_t)w_slots * (limbs * 8 + tables))
      return fail(KAD_ENOMEM, "no HBM left for the wide-count arena (%llu limbs per slot needed)",
                  (unsigned long long)want);
  } else {
    // Counts past 128 bits: at most as many slots as the sampler slots, as can be resident
    // and as 80% of the memory left allows, each with an arena that holds
    // any sample of the graph when that is at most WIDE_TIER1_LIMBS (or kad_ctx_set_wide's
    // size), else of that size, grown to what the memory gives.  Samples that outgrow it
    // are sampled again by a second pass: fewer slots with arenas of the worst case (at
    // most WIDE_MAX_LIMBS, at least the whole first-pass memory) carved from the same memory.
    const uint64_t A = left / 10 * 8;
    const uint64_t worst = std::max(wide_limbs_worst(g), ovc == 0 ? want : (uint64_t)0);
    const uint64_t target = ctx->w_user_limbs ? ctx->w_user_limbs : WIDE_TIER1_LIMBS;
    const uint64_t lim1 = std::min(worst, target);
    uint32_t most = std::min<uint32_t>(wide_slot_count(ctx), (uint32_t)ctx->wide_per_cu * ctx->cus);
    if (ctx->w_user_slots) most = std::min(most, ctx->w_user_slots);
    w_slots = (uint32_t)std::min<uint64_t>(most, A / (lim1 * 8 + tables));
    if (w_slots == 0)
      return fail(KAD_ENOMEM, "no HBM left for the wide-count arena (%llu limbs per slot needed)",
                  (unsigned long long)lim1);
    limbs = ctx->w_user_limbs
                ? lim1
                : std::min(worst, std::max(lim1, std::min<uint64_t>(
                                                     WIDE_MAX_LIMBS,
                                                     (A - (uint64_t)w_slots * tables) / 8 / w_slots)));
    if (limbs < worst) {
      const uint64_t total = (uint64_t)w_slots * limbs;
      w_slots2 = (uint32_t)std::max<uint64_t>(1, total / std::min(worst, WIDE_MAX_LIMBS));
      limbs2 = total / w_slots2;
    }
  }
  HIP_TRY(ctx->w_arena.ensure((size_t)w_slots * limbs));
  HIP_TRY(ctx->w_lv.ensure((size_t)w_slots * 2 * max_lev * 4));
  HIP_TRY(ctx->w_lbase.ensure((size_t)w_slots * 2 * max_lev));
  ctx->w_slots = w_slots;
  ctx->w_slots2 = w_slots2;
  ctx->w_max_lev = max_lev;
  ctx->w_arena_limbs = limbs;
  ctx->w_arena_limbs2 = limbs2;
  ctx->w_big = big;
  return KAD_OK;
}

int overflow_class(const kad_graph *g, uint32_t vd, bool vd_from_library) {
  if (!vd_from_library) return 1;
  if (vd <= 2 || g->maxdeg <= 1) return 0;
  // a path count is at most maxdeg^(levels), and levels < VD
  const double bits = (double)(vd - 1) * std::log2((double)g->maxdeg);
  if (bits < 127.0) return 0;
  if (vd >= 256 && g->arcs >= 3ull * g->n) return 2;
  return 1;
}

WideState wide_view(const kad_ctx *ctx) {
  WideState w;
  w.slots = std::min(ctx->w_slots, wide_slot_count(ctx));
  w.max_lev = ctx->w_max_lev;
  w.arena_limbs = ctx->w_arena_limbs;
  w.arena = ctx->w_arena.p;
  w.lv = ctx->w_lv.p;
  w.lbase = ctx->w_lbase.p;
  return w;
}

WideState wide_view2(const kad_ctx *ctx) {
  WideState w = wide_view(ctx);
  w.slots = std::min(ctx->w_slots2, w.slots);
  w.arena_limbs = ctx->w_arena_limbs2;
  return w;
}

kad_status launch_wide(kad_ctx *ctx, const GraphDev &g, uint64_t seed, uint32_t phase,
                       uint64_t first, const SampleSeg *segs, uint32_t nseg, uint32_t count,
                       bool all, const uint32_t *list, const uint32_t *list_count,
                       uint32_t *work, uint32_t *list2, const SampleOut &out,
                       hipStream_t stream, uint32_t slot0, const BatchDesc *bd) {
  if (count == 0) return KAD_OK;
  if (ctx->w_slots == 0) return fail(KAD_EINVAL, "internal: wide-count arena not allocated");
  // with slot tables the wide-count kernel has a pool of its own, which the wide passes of
  // one run take in turn (each waits for the previous one: they share the arena)
  const SlotState sv = wide_slot_view(ctx, ctx->slot_hbits ? 0u : slot0);
  WideState wv = wide_view(ctx);
  wv.slots = std::min(wv.slots, sv.slots);  // one dense slot per wide-count workgroup
  const bool two = ctx->w_slots2 > 0 && list2;
  SampleOut o1 = out, o2 = out;  // the first pass lists the samples its arenas cannot hold
  o1.fix_list = two ? list2 : nullptr;
  o1.fix_count = two ? work + 1 : nullptr;
  o2.fix_list = nullptr;
  o2.fix_count = nullptr;
  HIP_TRY(launch_wide_fix(g, seed, phase, first, segs, nseg, sv, wv, count, all, list,
                          list_count, work, o1, stream, bd));
  if (two) {
    WideState w2 = wide_view2(ctx);
    w2.slots = std::min(w2.slots, sv.slots);
    HIP_TRY(launch_wide_fix(g, seed, phase, first, segs, nseg, sv, w2, count, false, list2,
                            work + 1, work + 2, o2, stream, bd));
  }
  return KAD_OK;
}

LaunchShape graph_shape(const kad_graph *g) {
  if (g->shape_set) return g->shape;
  return LaunchShape{};
}

uint32_t launch_grid(const kad_ctx *ctx, const LaunchShape &shape, uint64_t count, uint32_t slot0) {
  int per_cu = 1;
  for (int j = 0; j < 3; ++j)
    if (SAMPLER_BLOCKS[j] == shape.block) per_cu = sampler_per_cu(ctx, shape.block);
  const uint64_t resident = (uint64_t)ctx->cus * (uint64_t)per_cu;
  const uint64_t slots = ctx->slots > slot0 ? ctx->slots - slot0 : 0;
  return (uint32_t)std::min<uint64_t>(std::min<uint64_t>(slots, resident), count);
}

SlotState slot_view(const kad_ctx *ctx, uint32_t slot0) {
  SlotState st;
  const size_t n = ctx->slot_hbits ? (size_t)1 << ctx->slot_hbits : ctx->slot_n;
  st.slots = ctx->slots > slot0 ? ctx->slots - slot0 : 0;
  st.n = (uint32_t)n;
  st.pi_cap = PI_CAP;
  st.rec = ctx->rec.p + (size_t)slot0 * n * REC_WORDS;
  st.visit = ctx->visit.p + (size_t)slot0 * n;
  st.pi = ctx->pi.p + (size_t)slot0 * PI_CAP;
  st.hbits = ctx->slot_hbits;
  st.vh = ctx->slot_hbits ? ctx->vh.p + (size_t)slot0 * n : nullptr;
  return st;
}

int sampler_per_cu(const kad_ctx *ctx, int block) {
  for (int j = 0; j < 3; ++j)
    if (SAMPLER_BLOCKS[j] == block)
      return ctx->slot_hbits ? ctx->blocks_per_cu_tab[j] : ctx->blocks_per_cu[j];
  return 1;
}

uint32_t wide_slot_count(const kad_ctx *ctx) {
  return ctx->slot_hbits ? ctx->wpool : ctx->slots;
}

SlotState wide_slot_view(const kad_ctx *ctx, uint32_t slot0) {
  if (!ctx->slot_hbits) return slot_view(ctx, slot0);
  SlotState st;
  const size_t n = ctx->slot_n;
  st.slots = ctx->wpool > slot0 ? ctx->wpool - slot0 : 0;
  st.n = ctx->slot_n;
  st.pi_cap = PI_CAP;
  st.rec = ctx->wrec.p + (size_t)slot0 * n * REC_WORDS;
  st.visit = ctx->wvisit.p + (size_t)slot0 * n;
  st.pi = ctx->wpi.p + (size_t)slot0 * PI_CAP;
  return st;
}

void node_outputs(uint32_t n, const uint64_t *cnt, uint64_t tau, uint64_t omega, bool rule,
                  double eps, const double *L_l, const double *L_u,
                  const std::vector<uint32_t> &grp_of, double *bc, double *lo, double *hi) {
  const double T = (double)tau, W = (double)omega;
  // f and g depend on (count, L_l, L_u) only: memoise per (group, count)
  struct Memo {
    uint64_t c;
    uint32_t grp;
    bool used;
    double f, g;
  };
  const bool grouped = grp_of.size() == n;
  parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned) {
    std::vector<Memo> memo(rule && grouped ? 16384 : 0, Memo{0, 0, false, 0.0, 0.0});
    for (uint32_t v = vb; v < ve; ++v) {
      bc[v] = (double)cnt[v] / T;
      if (rule) {
        double f, g;
        if (grouped) {
          const uint32_t gv = grp_of[v];
          Memo &m = memo[(uint32_t)((cnt[v] * 0x9E3779B97F4A7C15ULL ^ (uint64_t)gv * 0xC2B2AE3D27D4EB4FULL) >> 50)];
          if (!(m.used && m.c == cnt[v] && m.grp == gv))
            m = Memo{cnt[v], gv, true, bound_f(bc[v], L_l[v], W, T), bound_g(bc[v], L_u[v], W, T)};
          f = m.f;
          g = m.g;
        } else {
          f = bound_f(bc[v], L_l[v], W, T);
          g = bound_g(bc[v], L_u[v], W, T);
        }
        lo[v] = bc[v] - f;
        hi[v] = bc[v] + g;
      } else {
        lo[v] = bc[v] - eps;
        hi[v] = bc[v] + eps;
      }
    }
  });
}

void node_outputs_pilot(uint32_t n, const uint64_t *cnt, uint64_t tau, uint64_t omega, bool rule,
                        double eps, const uint64_t *count0, const std::vector<uint32_t> &cgrp,
                        const std::vector<double> &gL_l, const std::vector<double> &gL_u,
                        double *bc, double *lo, double *hi, uint64_t *count_out,
                        const std::function<void(uint32_t)> &wait_to) {
  const double T = (double)tau, W = (double)omega;
  struct Memo {
    uint64_t c;
    uint32_t grp;
    bool used;
    double f, g;
  };
  // one pass over the nodes: the caller's counts, b~ and the two bounds
  parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned) {
    thread_local std::vector<Memo> memo;  // kept by each worker: no fresh pages per call
    if (rule) memo.assign(16384, Memo{0, 0, false, 0.0, 0.0});
    if (wait_to) wait_to(ve);  // the counts of [0, ve) have landed
    for (uint32_t v = vb; v < ve; ++v) {
      const uint64_t c = cnt[v];
      if (count_out) count_out[v] = c;
      const double b = (double)c / T;
      bc[v] = b;
      if (rule) {
        const uint32_t gv = cgrp[count0[v]];
        Memo &m = memo[(uint32_t)((c * 0x9E3779B97F4A7C15ULL ^ (uint64_t)gv * 0xC2B2AE3D27D4EB4FULL) >> 50)];
        if (!(m.used && m.c == c && m.grp == gv))
          m = Memo{c, gv, true, bound_f(b, gL_l[gv], W, T), bound_g(b, gL_u[gv], W, T)};
        lo[v] = b - m.f;
        hi[v] = b + m.g;
      } else {
        lo[v] = b - eps;
        hi[v] = b + eps;
      }
    }
  });
}

// Sort x ascending on the worker threads: chunks sorted at once, then merged in pairs.
static void parallel_sort(std::vector<double> &x) {
  const size_t N = x.size();
  const unsigned K = std::min<unsigned>(kad::worker_count(), (unsigned)std::max<size_t>(1, N >> 16));
  if (K <= 1) {
    std::sort(x.begin(), x.end());
    return;
  }
  std::vector<size_t> cut(K + 1);
  for (unsigned c = 0; c <= K; ++c) cut[c] = N * c / K;
  kad::parallel_tasks(K, [&](unsigned c) { std::sort(x.begin() + cut[c], x.begin() + cut[c + 1]); });
  std::vector<double> tmp(N);
  std::vector<double> *src = &x, *dst = &tmp;
  for (unsigned w = 1; w < K; w *= 2) {  // runs of w chunks merged into runs of 2w
    const unsigned pairs = (K + 2 * w - 1) / (2 * w);
    kad::parallel_tasks(pairs, [&](unsigned p) {
      const size_t a = cut[std::min(K, 2 * w * p)], b = cut[std::min(K, 2 * w * p + w)],
                   e = cut[std::min(K, 2 * w * (p + 1))];
      std::merge(src->begin() + a, src->begin() + b, src->begin() + b, src->begin() + e,
                 dst->begin() + a);
    });
    std::swap(src, dst);
  }
  if (src != &x) x.swap(tmp);
}

// The nodes whose rank interval can reach the top k, with their rank intervals
// (rank_lo = 1 + #{w != v: lo(w) >= hi(v)}, rank_hi = #{w: hi(w) > lo(v)}), ordered by count
// descending, id ascending.  Without sorting all n bounds: rank_lo(v) <= k needs hi(v) above
// the (k+1)-th largest lower bound (else the k+1 largest lower bounds all reach hi(v)), and
// then every lower bound that reaches hi(v) is among the k largest; rank_hi of a selected
// node counts upper bounds above the selection's smallest lower bound only.  Loose bounds
// can select every node, so the output order comes from a counting sort by count when the
// counts are small (the selection is in id order and the sort is stable), and the rank_hi
// searches and the sort of the upper bounds run on the worker threads.
void topk_select(uint32_t n, uint32_t k, const uint64_t *cnt, const double *lo, const double *hi,
                 std::vector<uint32_t> &sel, std::vector<uint32_t> &rlo_sel,
                 std::vector<uint32_t> &rhi_sel) {
  sel.clear();
  rlo_sel.clear();
  rhi_sel.clear();
  if (n == 0) return;
  const uint32_t m = (uint32_t)std::min<uint64_t>(n, (uint64_t)k + 1);
  // The loops over the nodes run in ranges on the worker threads, each range's results
  // written at its offset in arrays sized by a counting pass (the selection stays in id
  // order).  parallel_ranges splits n the same way every time, so the passes agree.
  const unsigned nw = kad::worker_count();
  // the m largest lower bounds: each range's m largest, then the m largest of those
  std::vector<std::vector<double>> ptop(nw);
  kad::parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
    std::vector<double> &pt = ptop[w];
    pt.assign(lo + vb, lo + ve);
    if (pt.size() > m) {
      std::nth_element(pt.begin(), pt.begin() + (m - 1), pt.end(), std::greater<double>());
      pt.resize(m);
    }
  });
  std::vector<double> top;
  for (auto &pt : ptop) top.insert(top.end(), pt.begin(), pt.end());
  std::nth_element(top.begin(), top.begin() + (m - 1), top.end(), std::greater<double>());
  top.resize(m);
  std::sort(top.begin(), top.end(), std::greater<double>());  // the m largest, descending
  const bool everyone = (uint64_t)k + 1 > n;  // all lower bounds are in `top`
  const double floor_lo = top[m - 1];
  // rank_lo(v) - 1 = #{w != v: lo(w) >= hi(v)} when it is below k, else 0
  auto rank_lo_of = [&](uint32_t v) -> uint32_t {
    if (!everyone && !(hi[v] > floor_lo)) return 0;
    // #{w: lo(w) >= hi(v)}: the prefix of `top` that is >= hi(v)
    size_t ge = std::upper_bound(top.begin(), top.end(), hi[v], std::greater<double>()) -
                top.begin();
    if (lo[v] >= hi[v]) --ge;
    return 1 + ge <= k ? (uint32_t)(1 + ge) : 0u;
  };
  std::vector<uint32_t> at(nw + 1, 0);
  kad::parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
    uint32_t c = 0;
    for (uint32_t v = vb; v < ve; ++v) c += rank_lo_of(v) != 0;
    at[w + 1] = c;
  });
  for (unsigned w = 0; w < nw; ++w) at[w + 1] += at[w];
  const uint32_t S = at[nw];
  if (S == 0) return;
  sel.resize(S);
  std::vector<uint32_t> rl(S);
  kad::parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
    uint32_t o = at[w];
    for (uint32_t v = vb; v < ve; ++v) {
      const uint32_t r = rank_lo_of(v);
      if (r) {
        sel[o] = v;
        rl[o++] = r;
      }
    }
  });
  double t = lo[sel[0]];
  uint64_t cmax = 0;
  for (uint32_t v : sel) {
    t = std::min(t, lo[v]);
    cmax = std::max(cmax, cnt[v]);
  }
  // the upper bounds above t, gathered the same way
  std::vector<uint32_t> ua(nw + 1, 0);
  kad::parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
    uint32_t c = 0;
    for (uint32_t v = vb; v < ve; ++v) c += hi[v] > t;
    ua[w + 1] = c;
  });
  for (unsigned w = 0; w < nw; ++w) ua[w + 1] += ua[w];
  std::vector<double> up(ua[nw]);
  kad::parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
    uint32_t o = ua[w];
    for (uint32_t v = vb; v < ve; ++v)
      if (hi[v] > t) up[o++] = hi[v];
  });
  parallel_sort(up);
  // idx[q]: the position in sel of the q-th node in output order
  std::vector<uint32_t> idx(S);
  if (cmax <= 4ull * S + 1024) {
    std::vector<uint32_t> pos(cmax + 2, 0);  // bucket cmax - c holds count c
    for (uint32_t q = 0; q < S; ++q) pos[cmax - cnt[sel[q]] + 1]++;
    for (uint64_t b = 1; b <= cmax + 1; ++b) pos[b] += pos[b - 1];
    for (uint32_t q = 0; q < S; ++q) idx[pos[cmax - cnt[sel[q]]]++] = q;
  } else {
    for (uint32_t q = 0; q < S; ++q) idx[q] = q;
    std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
      const uint32_t x = sel[a], y = sel[b];
      return cnt[x] != cnt[y] ? cnt[x] > cnt[y] : x < y;
    });
  }
  std::vector<uint32_t> sorted(S);
  rlo_sel.resize(S);
  rhi_sel.resize(S);
  kad::parallel_ranges(S, [&](uint32_t qb, uint32_t qe, unsigned) {
    for (uint32_t q = qb; q < qe; ++q) {
      const uint32_t v = sel[idx[q]];
      sorted[q] = v;
      rlo_sel[q] = rl[idx[q]];
      rhi_sel[q] = (uint32_t)(up.end() - std::upper_bound(up.begin(), up.end(), lo[v]));
    }
  });
  sel.swap(sorted);
}

uint64_t run_items(const kad_graph *g, uint32_t target) {
  if (target == KAD_TARGET_EDGES) return g->directed ? g->arcs : g->arcs / 2;
  return g->n;
}

kad_status graph_edge_ids(kad_graph *g, const uint32_t **d_eid) {
  *d_eid = nullptr;
  if (g->directed) return KAD_OK;
  std::lock_guard<std::mutex> lk(g->eid_mu);
  if (!g->eid_ready) {
    std::vector<uint32_t> &eid = g->eid;
    eid.assign(g->arcs, 0);
    uint32_t next = 0;
    for (uint32_t u = 0; u < g->n; ++u)
      for (uint32_t e = g->row[u]; e < g->row[u + 1]; ++e) {
        const uint32_t v = g->col[e];
        if (v < u) continue;
        const uint32_t *b = g->col.data() + g->row[v], *en = g->col.data() + g->row[v + 1];
        const uint32_t back = (uint32_t)(std::lower_bound(b, en, u) - g->col.data());
        eid[e] = next;
        eid[back] = next;
        next++;
      }
    HIP_TRY(hipSetDevice(g->ctx->device));
    HIP_TRY(hipMalloc((void **)&g->d_eid, std::max<size_t>(g->arcs, 1) * 4));
    if (g->arcs)
      HIP_TRY(hipMemcpy(g->d_eid, eid.data(), (size_t)g->arcs * 4, hipMemcpyHostToDevice));
    g->bytes += g->arcs * 4;
    g->ctx->used_graphs += g->arcs * 4;
    g->eid_ready = true;
  }
  *d_eid = g->d_eid;
  return KAD_OK;
}

kad_status validate_params(const kad_graph *g, const kad_params *p) {
  if (p->target != KAD_TARGET_NODES && p->target != KAD_TARGET_EDGES)
    return fail(KAD_EINVAL, "target must be KAD_TARGET_NODES or KAD_TARGET_EDGES");
  if (!(p->epsilon > 0 && p->epsilon < 1)) return fail(KAD_EINVAL, "epsilon must be in (0,1)");
  if (!(p->delta > 0 && p->delta < 1)) return fail(KAD_EINVAL, "delta must be in (0,1)");
  if (p->mode != KAD_ALL_NODES && p->mode != KAD_TOPK) return fail(KAD_EINVAL, "bad mode");
  const uint64_t items = run_items(g, p->target);
  if (items == 0) return fail(KAD_EINVAL, "the graph has no edges");
  if (items > (uint64_t)MAX_HIT_TILES_PUBLIC * HIT_TILE_IDS)
    return fail(KAD_EINVAL, "runs over more than %u items are not supported",
                MAX_HIT_TILES_PUBLIC * HIT_TILE_IDS);
  if (p->mode == KAD_TOPK && (p->k < 1 || p->k > items))
    return fail(KAD_EINVAL, "k must be in [1, items]");
  if (p->schedule > KAD_SCHEDULE_HOEFFDING) return fail(KAD_EINVAL, "unknown schedule");
  if (p->c < 0) return fail(KAD_EINVAL, "c must be positive (or 0 for the default)");
  if (!(p->balance_eps >= 0 && p->balance_eps < 0.5))
    return fail(KAD_EINVAL, "balance_eps must be in (0, 0.5) (or 0 for the default)");
  return KAD_OK;
}


// Record the launches `fn` makes on the stream it is given into bg, unless bg already
// holds a recording with this key.
kad_status record_chain(kad_ctx *ctx, BatchGraph &bg, const ChainKey &key,
                        const std::function<kad_status(hipStream_t)> &fn) {
  if (bg.exec && bg.key == key.v) return KAD_OK;
  bg.release();
  if (!ctx->cstream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cstream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(ctx->cstream, hipStreamCaptureModeThreadLocal));
  const kad_status st = fn(ctx->cstream);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cstream, &gr);
  if (st != KAD_OK || e != hipSuccess || !gr) {
    if (gr) (void)hipGraphDestroy(gr);
    if (st != KAD_OK) return st;
    return fail(KAD_EDEVICE, "recording a batch chain failed: %s", hipGetErrorString(e));
  }
  bg.graph = gr;
  const hipError_t ei = hipGraphInstantiate(&bg.exec, gr, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    bg.release();
    return fail(KAD_EDEVICE, "instantiating a batch chain failed: %s", hipGetErrorString(ei));
  }
  bg.key = key.v;
  bg.records++;
  ctx->chain_records++;
  return KAD_OK;
}

}  // namespace kad

namespace {

using kad::DevBuf;
using kad::PinBuf;
using kad::OutSet;
using kad::fail;
using kad::PI_CAP;
using kad::DEFAULT_BATCH;
using kad::dev_view;
using kad::graph_vd;

// Rows sorted strictly ascending, heads in range, no self-loops.  The row pointers are
// checked first, so that no row is read before its bounds are known to lie within the
// arcs; the rows before the first bad pointer are then checked in ranges on the worker
// threads.  The error reported is that of the first bad node.
kad_status check_rows(uint32_t n, uint64_t arcs, const uint32_t *row, const uint32_t *col,
                      const char *what) {
  if (row[0] != 0 || row[n] != arcs) return fail(KAD_EINVAL, "%s: row_ptr[0] must be 0 and row_ptr[n] = arcs", what);
  uint32_t d = n;  // the first node whose row pointer decreases or passes the arcs
  for (uint32_t v = 0; v < n; ++v)
    if (row[v + 1] < row[v] || row[v + 1] > arcs) {
      d = v;
      break;
    }
  // per range: the first bad row (kind 1 head out of range, 2 self-loop, 3 not ascending)
  struct Bad { uint32_t v = UINT32_MAX, kind = 0, x = 0; };
  std::vector<Bad> bad(kad::worker_count());
  kad::parallel_ranges(d, [&](uint32_t lo, uint32_t hi, unsigned w) {
    Bad b;
    for (uint32_t v = lo; v < hi && b.kind == 0; ++v)
      for (uint32_t e = row[v]; e < row[v + 1]; ++e) {
        const uint32_t x = col[e];
        const uint32_t k = x >= n ? 1u : x == v ? 2u : (e > row[v] && col[e - 1] >= x) ? 3u : 0u;
        if (k) {
          b = {v, k, x};
          break;
        }
      }
    bad[w] = b;
  });
  const Bad b = *std::min_element(bad.begin(), bad.end(),
                                  [](const Bad &a, const Bad &c) { return a.v < c.v; });
  switch (b.kind) {
    case 1: return fail(KAD_EINVAL, "%s: node %u has out-of-range neighbour %u", what, b.v, b.x);
    case 2: return fail(KAD_EINVAL, "%s: self-loop at node %u", what, b.v);
    case 3: return fail(KAD_EINVAL, "%s: row %u is not strictly ascending", what, b.v);
    default: break;
  }
  if (d < n) {
    if (row[d + 1] < row[d]) return fail(KAD_EINVAL, "%s: row_ptr decreases at node %u", what, d);
    return fail(KAD_EINVAL, "%s: row_ptr[%u] passes the arc count", what, d + 1);
  }
  return KAD_OK;
}

// The in-rows of (row, col): for each node x, the tails of the arcs into x, ascending.
// The tails are split into K chunks of about equal arc counts, one per worker thread;
// each chunk counts its heads, a prefix over (head, chunk) gives every chunk its place in
// each in-row, and each chunk then writes its arcs in tail order, so every in-row comes
// out ascending.  The per-chunk counts take 4 n bytes per chunk (K is cut to keep them
// within 1 GiB).
void transpose(uint32_t n, const std::vector<uint32_t> &row, const std::vector<uint32_t> &col,
               std::vector<uint32_t> &trow, std::vector<uint32_t> &tcol) {
  const uint64_t m = col.size();
  const uint64_t by_mem = std::max<uint64_t>(1, (1ull << 28) / std::max<uint32_t>(n, 1));
  const unsigned K = (unsigned)std::min<uint64_t>(
      {(uint64_t)kad::parallel_threads((uint32_t)std::min<uint64_t>(m, UINT32_MAX)),
       (uint64_t)kad::worker_count(), by_mem});
  std::vector<uint32_t> cut(K + 1);  // chunk k: tails [cut[k], cut[k + 1])
  for (unsigned k = 0; k < K; ++k)
    cut[k] = (uint32_t)(std::lower_bound(row.begin(), row.end(), (uint32_t)(m * k / K)) - row.begin());
  cut[K] = n;
  std::unique_ptr<uint32_t[]> cnt(new uint32_t[(size_t)K * n]);  // [chunk][head]
  kad::parallel_tasks(K, [&](unsigned k) {
    uint32_t *c = cnt.get() + (size_t)k * n;
    std::fill(c, c + n, 0u);
    for (uint32_t e = row[cut[k]]; e < row[cut[k + 1]]; ++e) c[col[e]]++;
  });
  trow.assign((size_t)n + 1, 0);
  kad::parallel_ranges(n, [&](uint32_t lo, uint32_t hi, unsigned) {
    for (uint32_t x = lo; x < hi; ++x) {
      uint32_t s = 0;
      for (unsigned k = 0; k < K; ++k) {
        uint32_t &c = cnt[(size_t)k * n + x];
        const uint32_t t = c;
        c = s;  // chunk k's first place in in-row x, counted from the row's start
        s += t;
      }
      trow[x + 1] = s;
    }
  });
  for (uint32_t x = 0; x < n; ++x) trow[x + 1] += trow[x];
  tcol.resize(m);
  kad::parallel_tasks(K, [&](unsigned k) {
    uint32_t *c = cnt.get() + (size_t)k * n;
    for (uint32_t v = cut[k]; v < cut[k + 1]; ++v)
      for (uint32_t e = row[v]; e < row[v + 1]; ++e) {
        const uint32_t x = col[e];
        tcol[trow[x] + c[x]++] = v;
      }
  });
}

hipStream_t pick_stream(kad_ctx *ctx, void *s) { return s ? (hipStream_t)s : ctx->stream; }

// Size the slot state, the wide-count arena and both output sets for graph g (overflow
// class ovc) and `batch` samples of path stride `stride`.
kad_status ensure_capacity(kad_ctx *ctx, const kad_graph *g, int ovc, uint32_t batch,
                           uint32_t stride, uint64_t items = 0, bool edges = false) {
  const uint32_t n = g->n;
  if (items == 0) items = n;  // the counters: one per node, or per edge
  kad_status st = kad::ensure_slots(ctx, n);
  if (st) return st;
  if ((st = kad::ensure_wide(ctx, g, ovc))) return st;
  for (OutSet &o : ctx->outs) {
    if ((st = o.ensure(batch, stride, ctx->rstream))) return st;
    if (edges && (st = o.ensure_edges(o.cap, o.stride + 1))) return st;
  }
  HIP_TRY(ctx->work.ensure(kad::WORK_WORDS));
  HIP_TRY(ctx->work2.ensure(kad::WORK_WORDS));
  HIP_TRY(ctx->count.ensure(items));
  HIP_TRY(ctx->h_count.ensure(items));
  // hit-reduction bins: room in every tile for all the hits of one reduction call
  // (fixed layout), or, when that would pass 1 GiB (long paths), one array sized by the
  // hits with a counting pass first (compact layout).  A path of len nodes has len - 2
  // interior nodes and len - 1 edges.
  const uint64_t tiles = (items + kad::HIT_TILE_IDS - 1) / kad::HIT_TILE_IDS;
  if (tiles > kad::MAX_HIT_TILES_PUBLIC)
    return fail(KAD_EINVAL, "more than %u counters are not supported by the hit reduction",
                kad::MAX_HIT_TILES_PUBLIC * kad::HIT_TILE_IDS);
  const uint32_t rstride = ctx->outs[0].stride + (edges ? 1 : 0);
  const uint64_t cap = (uint64_t)ctx->outs[0].cap * std::max<uint32_t>(rstride - 2, 1);
  const bool compact = tiles * cap * 4 > (1ull << 30);
  const uint64_t want = compact ? cap : tiles * cap;
  if (cap > ctx->bins_cap || want > ctx->bins.n || compact != ctx->bins_compact) {
    ctx->bins.release();
    HIP_TRY(ctx->bins.ensure(want));
    ctx->bins_cap = cap;
    ctx->bins_compact = compact;
  }
  if (ctx->bin_count.n == 0) {
    HIP_TRY(ctx->bin_count.ensure(kad::MAX_HIT_TILES_PUBLIC));
    HIP_TRY(ctx->tile_start.ensure(kad::MAX_HIT_TILES_PUBLIC));
    HIP_TRY(ctx->tile_fill.ensure(kad::MAX_HIT_TILES_PUBLIC));
    HIP_TRY(hipMemset(ctx->bin_count.p, 0, kad::MAX_HIT_TILES_PUBLIC * 4));
    HIP_TRY(hipMemset(ctx->tile_fill.p, 0, kad::MAX_HIT_TILES_PUBLIC * 4));
  }
  return KAD_OK;
}

kad::HitScratch hit_scratch(kad_ctx *ctx) {
  kad::HitScratch h;
  h.bins = ctx->bins.p;
  h.cap = ctx->bins_cap;
  h.bin_count = ctx->bin_count.p;
  if (ctx->bins_compact) {
    h.tile_start = ctx->tile_start.p;
    h.tile_fill = ctx->tile_fill.p;
  }
  return h;
}

// Enqueue the sampler on ids [first, first+count) into output set `set`, then the
// copies of its flags and arcs (and, when timing, nodes and lengths) to the host
// mirrors; nothing waits.
// ovc: the graph's overflow class (kad::overflow_class): 0 = 128-bit counts always
// suffice, 1 = resample overflowed samples wide, 2 = sample everything wide.
// slot0, work: the launch's sampler slots start at slot0 and its work counter is *work
// (ctx->work when null), so that two launches on different streams may overlap.
// wide_after: the wide-count fix (which shares one arena across launches) waits for it.
kad_status launch_batch(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                        uint64_t first, uint32_t count, uint32_t stride, int set,
                        hipStream_t stream, int ovc, uint32_t slot0 = 0, uint32_t *work = nullptr,
                        hipEvent_t wide_after = nullptr, bool edges = false,
                        const uint32_t *edge_ids = nullptr) {
  OutSet &o = ctx->outs[set];
  kad_status st = KAD_OK;
  uint32_t *wk = work ? work : ctx->work.p;  // the launch's counters (kad::WORK_WORDS)
  HIP_TRY(hipEventRecord(o.k0, stream));
  HIP_TRY(kad::launch_zero_u32(wk, kad::WORK_WORDS, stream));
  if (ovc == 2) {
    if (wide_after) HIP_TRY(hipStreamWaitEvent(stream, wide_after, 0));
    st = kad::launch_wide(ctx, dev_view(g), seed, phase, first, nullptr, 0, count, true, nullptr,
                          nullptr, wk + 2, o.fix_list2.p, o.view(stride), stream, slot0);
    if (st) return st;
    HIP_TRY(hipEventRecord(o.k1, stream));
    o.h_nwide.p[0] = count;
  } else {
    const kad::LaunchShape shape = kad::graph_shape(g);
    const uint32_t grid = kad::launch_grid(ctx, shape, count, slot0);
    HIP_TRY(kad::launch_sampler(dev_view(g), kad::slot_view(ctx, slot0), seed, phase, first,
                                count, wk, o.view(stride, wk + 1), grid, shape, stream));
    HIP_TRY(hipEventRecord(o.k1, stream));
    // the samples the sampler left (counts past 128 bits, more candidate edges than a slot
    // holds) are sampled again by the wide-count kernel; an empty list costs one short launch
    if (wide_after) HIP_TRY(hipStreamWaitEvent(stream, wide_after, 0));
    st = kad::launch_wide(ctx, dev_view(g), seed, phase, first, nullptr, 0, count, false,
                          o.fix_list.p, wk + 1, wk + 2, o.fix_list2.p, o.view(stride), stream,
                          slot0);
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(o.h_nwide.p, wk + 1, 4, hipMemcpyDeviceToHost, stream));
  }
  if (edges)  // the paths as edge ids, for the edge-hit reductions
    HIP_TRY(kad::launch_edge_paths(o.path.p, o.len.p, stride, count, g->d_row, g->d_col, edge_ids,
                                   o.epath.p, o.elen.p, stride + 1, stream));
  // the reductions need only the paths: they wait for this event, not for the mirrors
  // (a set is launched into again only after the host has waited for its mirrors)
  HIP_TRY(hipEventRecord(o.sampled, stream));
  HIP_TRY(hipMemcpyAsync(o.h_flags.p, o.flags.p, (size_t)count * 4, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(o.h_arcs.p, o.arcs.p, (size_t)count * 8, hipMemcpyDeviceToHost, stream));
  if (ctx->timing) {
    HIP_TRY(hipMemcpyAsync(o.h_nodes.p, o.nodes.p, (size_t)count * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(o.h_len.p, o.len.p, (size_t)count * 4, hipMemcpyDeviceToHost, stream));
  }
  HIP_TRY(hipEventRecord(o.copied, stream));
  return KAD_OK;
}

// ---------------------------------------------------------------- recorded batch chains
// The main-phase batch [first, first + count) of output set `set`, as launch_batch makes
// it (slots from 0, the context's work counters), by replaying the set's recorded sampling
// chain for batches of up to `cap` samples.  niv: the batch's check intervals (read by the
// reduction chain's descriptor, written by replay_reduce).
kad_status replay_sampling(kad_ctx *ctx, const kad_graph *g, int set, uint64_t seed,
                           uint32_t phase, uint64_t first, uint32_t count, uint32_t cap,
                           uint32_t stride, hipStream_t stream, int ovc, bool edges,
                           const uint32_t *edge_ids) {
  if (count == 0 || count > cap) return fail(KAD_EINVAL, "internal: batch of %u > %u", count, cap);
  if (ctx->w_slots == 0) return fail(KAD_EINVAL, "internal: wide-count arena not allocated");
  OutSet &o = ctx->outs[set];
  HIP_TRY(ctx->h_bd.ensure(4));
  HIP_TRY(ctx->d_bd.ensure(4));
  const kad::GraphDev gd = dev_view(g);
  const kad::LaunchShape shape = kad::graph_shape(g);
  const uint32_t grid = kad::launch_grid(ctx, shape, cap, 0);
  const kad::SlotState sv = kad::slot_view(ctx, 0), wsv = kad::wide_slot_view(ctx, 0);
  const kad::WideState wv = kad::wide_view(ctx), wv2 = kad::wide_view2(ctx);
  uint32_t *wk = ctx->work.p;  // the launch's counters (kad::WORK_WORDS)
  const kad::SampleOut so_list = o.view(stride, wk + 1), so = o.view(stride);
  kad::BatchDesc *hb = ctx->h_bd.p + set, *db = ctx->d_bd.p + set;
  kad::ChainKey key;
  key << 1 << set << gd << sv << wsv << wv << wv2 << so_list << o.fix_list2.p << shape.block
      << shape.small_exp << grid << cap << stride << ovc << edges << edge_ids << o.epath.p
      << o.elen.p << o.h_flags.p << o.h_arcs.p << o.h_nwide.p << wk << hb << db;
  kad_status st = kad::record_chain(ctx, ctx->bgraph[set], key, [&](hipStream_t s) -> kad_status {
    HIP_TRY(kad::launch_copy_u64(reinterpret_cast<uint64_t *>(db),
                                 reinterpret_cast<const uint64_t *>(hb),
                                 sizeof(kad::BatchDesc) / 8, s));
    HIP_TRY(kad::launch_zero_u32(wk, kad::WORK_WORDS, s));
    kad_status ws;
    if (ovc == 2) {
      if ((ws = kad::launch_wide(ctx, gd, 0, 0, 0, nullptr, 0, cap, true, nullptr, nullptr,
                                 wk + 2, o.fix_list2.p, so, s, 0, db)))
        return ws;
    } else {
      HIP_TRY(kad::launch_sampler(gd, sv, 0, 0, 0, cap, wk, so_list, grid, shape, s, db));
      if ((ws = kad::launch_wide(ctx, gd, 0, 0, 0, nullptr, 0, cap, false, o.fix_list.p, wk + 1,
                                 wk + 2, o.fix_list2.p, so, s, 0, db)))
        return ws;
      HIP_TRY(kad::launch_copy_u32(o.h_nwide.p, wk + 1, 1, s));
    }
    if (edges)
      HIP_TRY(kad::launch_edge_paths(o.path.p, o.len.p, stride, cap, g->d_row, g->d_col,
                                     edge_ids, o.epath.p, o.elen.p, stride + 1, s, db));
    HIP_TRY(kad::launch_copy_u32(o.h_flags.p, o.flags.p, cap, s, db));
    HIP_TRY(kad::launch_copy_u64(o.h_arcs.p, o.arcs.p, cap, s, db));
    return KAD_OK;
  });
  if (st) return st;
  // the set's previous replay read this descriptor before its mirrors landed, and the
  // host has waited for those
  *hb = kad::BatchDesc{seed, first, count, phase, 0u, 0u, 0u, 0u};  // stride 0: the launch's own
  HIP_TRY(hipGraphLaunch(ctx->bgraph[set].exec, stream));
  ctx->bgraph[set].replays++;
  ctx->chain_replays++;
  if (ovc == 2) o.h_nwide.p[0] = count;
  HIP_TRY(hipEventRecord(o.sampled, stream));
  HIP_TRY(hipEventRecord(o.copied, stream));
  return KAD_OK;
}

// Every check interval of a batch of `count` samples of output set `set` reduced
// (launch_hit_batch) by replaying the set's recorded reduction chain for batches of up to
// `cap` samples; the snapshots land in snaps.
kad_status replay_reduce(kad_ctx *ctx, int set, const uint32_t *rpath, const uint32_t *rlen,
                         uint32_t rstride, uint32_t count, uint32_t cap, uint32_t per_iv,
                         uint32_t n, uint32_t ngroups, uint64_t *snaps, hipStream_t rs) {
  if (count == 0 || count > cap) return fail(KAD_EINVAL, "internal: batch of %u > %u", count, cap);
  HIP_TRY(ctx->h_bd.ensure(4));
  HIP_TRY(ctx->d_bd.ensure(4));
  kad::BatchDesc *hb = ctx->h_bd.p + 2 + set, *db = ctx->d_bd.p + 2 + set;
  kad::ChainKey key;
  key << 2 << set << rpath << rlen << rstride << cap << per_iv << n << ngroups << ctx->count.p
      << ctx->group.p << ctx->gmax.p << ctx->ivtmp.p << ctx->ivmax.p << snaps << hb << db;
  kad_status st = kad::record_chain(ctx, ctx->bgraph[2 + set], key, [&](hipStream_t s) -> kad_status {
    HIP_TRY(kad::launch_copy_u64(reinterpret_cast<uint64_t *>(db),
                                 reinterpret_cast<const uint64_t *>(hb),
                                 sizeof(kad::BatchDesc) / 8, s));
    HIP_TRY(kad::launch_hit_batch(rpath, rlen, rstride, cap, per_iv, n, ctx->count.p,
                                  ctx->group.p, ctx->gmax.p, ngroups, ctx->ivtmp.p,
                                  ctx->ivmax.p, snaps, s, db));
    return KAD_OK;
  });
  if (st) return st;
  // the previous replay of this chain is complete: the host waited for its snapshots
  *hb = kad::BatchDesc{0, 0, count, 0u, (count + per_iv - 1) / per_iv, 0u, 0u, 0u};
  HIP_TRY(hipGraphLaunch(ctx->bgraph[2 + set].exec, rs));
  ctx->bgraph[2 + set].replays++;
  ctx->chain_replays++;
  return KAD_OK;
}

// Wait for an event by polling: a run waits on many short GPU steps, and a blocking
// wait was seen to wake several hundred microseconds late.  After 2 ms of polling the
// wait blocks.
hipError_t wait_event(hipEvent_t ev) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2))
      return hipEventSynchronize(ev);
  }
}

// A stream's work so far, waited for with wait_event.
hipError_t wait_stream(kad_ctx *ctx, hipStream_t s) {
  hipEvent_t &ev = s == ctx->rstream ? ctx->ev_rs : (s == ctx->pstream ? ctx->ev_ps : ctx->ev_s);
  if (!ev) {
    const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  const hipError_t e = hipEventRecord(ev, s);
  if (e != hipSuccess) return e;
  return wait_event(ev);
}

// Timing within kad_run: the first main batch may run beside the pilot, so the run's
// sampler time is the union of its launches' event intervals (measured from a reference
// event recorded when the run starts), not their sum.
kad_status run_timing_begin(kad_ctx *ctx, hipStream_t s) {
  ctx->t_run_ref = false;
  if (!ctx->timing) return KAD_OK;
  if (!ctx->t_ref) HIP_TRY(hipEventCreate(&ctx->t_ref));
  HIP_TRY(hipEventRecord(ctx->t_ref, s));
  ctx->t_iv.clear();
  ctx->t_run_ref = true;
  return KAD_OK;
}
void run_timing_end(kad_ctx *ctx) {
  if (!ctx->t_run_ref) return;
  auto &iv = ctx->t_iv;
  std::sort(iv.begin(), iv.end());
  double busy = 0.0, lo = 0.0, hi = -1.0;
  for (const auto &x : iv) {
    if (x.first > hi) {
      if (hi > lo) busy += hi - lo;
      lo = x.first;
      hi = x.second;
    } else {
      hi = std::max(hi, (double)x.second);
    }
  }
  if (hi > lo) busy += hi - lo;
  ctx->t_seconds += busy * 1e-3;
  iv.clear();
  ctx->t_run_ref = false;
}

// Wait for a batch's mirrors, account its launch time, and reject flagged samples
// among the first `used` samples (samples past a stopping point do not matter).
kad_status finish_batch(kad_ctx *ctx, int set, uint32_t count, uint32_t used) {
  OutSet &o = ctx->outs[set];
  HIP_TRY(wait_event(o.copied));
  ctx->run_wide += o.h_nwide.p[0];
  if (ctx->timing) {
    if (ctx->t_run_ref) {  // a kad_run in progress: its launches may overlap; see run_busy
      float a = 0.f, b = 0.f;
      HIP_TRY(hipEventElapsedTime(&a, ctx->t_ref, o.k0));
      HIP_TRY(hipEventElapsedTime(&b, ctx->t_ref, o.k1));
      ctx->t_iv.emplace_back(a, b);
    } else {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, o.k0, o.k1));
      ctx->t_seconds += ms * 1e-3;
    }
    ctx->t_launches += 1;
    ctx->t_samples += count;
    ctx->t_wide += o.h_nwide.p[0];
    for (uint32_t k = 0; k < count; ++k) {
      ctx->t_arcs += o.h_arcs.p[k];
      ctx->t_nodes += o.h_nodes.p[k];
      ctx->t_hits += o.h_len.p[k] >= 2 ? o.h_len.p[k] - 2 : 0;
    }
  }
  for (uint32_t k = 0; k < used; ++k) {
    const uint32_t f = o.h_flags.p[k];
    if (f & kad::FLAG_OVERFLOW)
      return fail(KAD_EOVERFLOW, "a path count exceeded 128 bits (sample %u of the batch)", k);
    if (f & kad::FLAG_RNG) return fail(KAD_ERNG, "bounded draw rejected 64 times");
    if (f & kad::FLAG_CAPACITY)
      return fail(KAD_EOVERFLOW, "candidate-edge list or path outgrew its buffer (sample %u)", k);
  }
  return KAD_OK;
}

}  // namespace

extern "C" {

const char *kad_last_error(void) { return kad::g_error.c_str(); }

kad_status kad_ctx_create(int hip_device, uint64_t hbm_budget_bytes, kad_ctx **out) try {
  if (!out) return fail(KAD_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return fail(KAD_EDEVICE, "no HIP device available");
  if (hip_device < 0 || hip_device >= ndev) return fail(KAD_EDEVICE, "device %d does not exist", hip_device);
  std::unique_ptr<kad_ctx> c(new kad_ctx());
  c->device = hip_device;
  HIP_TRY(hipSetDevice(hip_device));
  HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&c->rstream, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&c->pstream, hipStreamNonBlocking));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
  c->cus = (uint32_t)prop.multiProcessorCount;
  for (int j = 0; j < 3; ++j) {
    c->blocks_per_cu[j] = kad::sampler_blocks_per_cu(kad::SAMPLER_BLOCKS[j], false);
    c->blocks_per_cu_tab[j] = kad::sampler_blocks_per_cu(kad::SAMPLER_BLOCKS[j], true);
  }
  c->wide_per_cu = kad::wide_blocks_per_cu();
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
  // the fixed scratch of kad_hit_counts_noalloc: its address on this device, looked up now
  // (with the device current) so that the call itself needs no runtime set-up
  HIP_TRY(kad::noalloc_scratch(&c->noalloc));
  *out = c.release();
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_destroy(kad_ctx *ctx) try {
  if (!ctx) return KAD_OK;
  (void)hipSetDevice(ctx->device);
  kad::destroy_engine(ctx->engine);  // waits for its work on the context's streams
  ctx->engine = nullptr;
  if (ctx->ev_s) (void)hipEventDestroy(ctx->ev_s);
  if (ctx->ev_rs) (void)hipEventDestroy(ctx->ev_rs);
  if (ctx->ev_ps) (void)hipEventDestroy(ctx->ev_ps);
  if (ctx->t_ref) (void)hipEventDestroy(ctx->t_ref);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  if (ctx->rstream) (void)hipStreamDestroy(ctx->rstream);
  if (ctx->pstream) (void)hipStreamDestroy(ctx->pstream);
  for (kad::BatchGraph &b : ctx->bgraph) b.release();
  if (ctx->cstream) (void)hipStreamDestroy(ctx->cstream);
  delete ctx;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_graph_create(kad_ctx *ctx, uint32_t n, uint64_t arcs, int directed,
                            const uint32_t *row_ptr, const uint32_t *col,
                            const uint32_t *rrow_ptr, const uint32_t *rcol, int mem,
                            kad_graph **out) try {
  if (!ctx || !out || !row_ptr || (!col && arcs)) return fail(KAD_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 2) return fail(KAD_EINVAL, "a graph needs at least 2 nodes");
  if (arcs >= (1ull << 32)) return fail(KAD_EINVAL, "arcs must be below 2^32");
  if (mem != KAD_MEM_HOST && mem != KAD_MEM_DEVICE) return fail(KAD_EINVAL, "bad mem kind");
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<kad_graph> g(new kad_graph());
  g->ctx = ctx;
  g->n = n;
  g->arcs = arcs;
  g->directed = directed != 0;
  g->row.resize((size_t)n + 1);
  g->col.resize(arcs);
  auto fetch = [&](std::vector<uint32_t> &dst, const uint32_t *src, size_t cnt) -> hipError_t {
    if (cnt == 0) return hipSuccess;
    if (mem == KAD_MEM_HOST) {
      memcpy(dst.data(), src, cnt * 4);
      return hipSuccess;
    }
    return hipMemcpy(dst.data(), src, cnt * 4, hipMemcpyDeviceToHost);
  };
  HIP_TRY(fetch(g->row, row_ptr, (size_t)n + 1));
  HIP_TRY(fetch(g->col, col, arcs));
  kad_status st = check_rows(n, arcs, g->row.data(), g->col.data(), "out-rows");
  if (st) return st;
  std::vector<uint32_t> trow, tcol;
  transpose(n, g->row, g->col, trow, tcol);
  if (!g->directed) {
    if (trow != g->row || tcol != g->col) return fail(KAD_EINVAL, "undirected graph is not symmetric");
  } else if (rrow_ptr && rcol) {
    g->rrow.resize((size_t)n + 1);
    g->rcol.resize(arcs);
    HIP_TRY(fetch(g->rrow, rrow_ptr, (size_t)n + 1));
    HIP_TRY(fetch(g->rcol, rcol, arcs));
    if (g->rrow != trow || g->rcol != tcol) return fail(KAD_EINVAL, "in-rows are not the transpose of the out-rows");
  } else {
    g->rrow.swap(trow);
    g->rcol.swap(tcol);
  }
  for (uint32_t v = 0; v < n; ++v) {
    g->maxdeg = std::max(g->maxdeg, g->row[v + 1] - g->row[v]);
    if (g->directed) g->maxdeg = std::max(g->maxdeg, g->rrow[v + 1] - g->rrow[v]);
  }
  const bool borrow = mem == KAD_MEM_DEVICE;
  const size_t rbytes = ((size_t)n + 1) * 4, cbytes = (size_t)arcs * 4;
  if (borrow) {
    g->d_row = const_cast<uint32_t *>(row_ptr);
    g->d_col = const_cast<uint32_t *>(col);
  } else {
    g->owns_fwd = true;
    HIP_TRY(hipMalloc((void **)&g->d_row, rbytes));
    HIP_TRY(hipMalloc((void **)&g->d_col, std::max<size_t>(cbytes, 4)));
    HIP_TRY(hipMemcpy(g->d_row, g->row.data(), rbytes, hipMemcpyHostToDevice));
    if (cbytes) HIP_TRY(hipMemcpy(g->d_col, g->col.data(), cbytes, hipMemcpyHostToDevice));
    g->bytes += rbytes + cbytes;
  }
  if (g->directed) {
    if (borrow && rrow_ptr && rcol) {
      g->d_rrow = const_cast<uint32_t *>(rrow_ptr);
      g->d_rcol = const_cast<uint32_t *>(rcol);
    } else {
      g->owns_rev = true;
      HIP_TRY(hipMalloc((void **)&g->d_rrow, rbytes));
      HIP_TRY(hipMalloc((void **)&g->d_rcol, std::max<size_t>(cbytes, 4)));
      HIP_TRY(hipMemcpy(g->d_rrow, g->rrow.data(), rbytes, hipMemcpyHostToDevice));
      if (cbytes) HIP_TRY(hipMemcpy(g->d_rcol, g->rcol.data(), cbytes, hipMemcpyHostToDevice));
      g->bytes += rbytes + cbytes;
    }
  }
  ctx->used_graphs += g->bytes;
  *out = g.release();
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_graph_destroy(kad_graph *g) try {
  if (!g) return KAD_OK;
  (void)hipSetDevice(g->ctx->device);
  if (g->owns_fwd) {
    (void)hipFree(g->d_row);
    (void)hipFree(g->d_col);
  }
  if (g->owns_rev) {
    (void)hipFree(g->d_rrow);
    (void)hipFree(g->d_rcol);
  }
  if (g->d_eid) (void)hipFree(g->d_eid);
  g->ctx->used_graphs -= std::min(g->ctx->used_graphs, g->bytes);
  delete g;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

// ---------------------------------------------------------------- host statistics

uint64_t kad_omega(double epsilon, double delta, uint32_t vd, double c) {
  return kad::omega_of(epsilon, delta, vd, c > 0 ? c : 0.5);
}
uint64_t kad_alpha(uint64_t omega) { return kad::alpha_of(omega); }

uint64_t kad_fixed_samples(uint32_t schedule, double epsilon, double delta, uint32_t vd,
                           uint32_t n, double c) {
  if (schedule == KAD_SCHEDULE_RK)  // ln(2/(2 delta)) = ln(1/delta): omega's form with 2 delta
    return kad::omega_of(epsilon, 2.0 * delta, vd, c > 0 ? c : 0.5);
  if (schedule == KAD_SCHEDULE_HOEFFDING)
    return (uint64_t)std::ceil(std::log(2.0 * (double)n / delta) / (2.0 * epsilon * epsilon));
  return 0;
}
uint64_t kad_default_interval(uint64_t omega) { return kad::interval_of(omega); }

kad_status kad_vertex_diameter(uint32_t n, uint64_t arcs, int directed, const uint32_t *row_ptr,
                               const uint32_t *col, const uint32_t *rrow_ptr,
                               const uint32_t *rcol, double exact_limit, uint32_t *vd,
                               uint32_t *exact) try {
  if (!vd || !exact || !row_ptr || (arcs && !col)) return fail(KAD_EINVAL, "NULL argument");
  if (directed && (!rrow_ptr || !rcol)) return fail(KAD_EINVAL, "directed graph needs in-rows");
  if (n == 0) return fail(KAD_EINVAL, "a graph needs at least one node");
  if (arcs >= (1ull << 32)) return fail(KAD_EINVAL, "arcs must be below 2^32");
  kad_status st = check_rows(n, arcs, row_ptr, col, "out-rows");
  if (!st && directed) st = check_rows(n, arcs, rrow_ptr, rcol, "in-rows");
  if (st) return st;
  bool ex = false;
  if (kad::vertex_diameter(n, arcs, row_ptr, col, directed ? rrow_ptr : row_ptr,
                           directed ? rcol : col, exact_limit, vd, &ex))
    return fail(KAD_EINVAL, "bad graph");
  *exact = ex ? 1u : 0u;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

double kad_bound_f(double btilde, double L, double omega, double tau) {
  return kad::bound_f(btilde, L, omega, tau);
}
double kad_bound_g(double btilde, double L, double omega, double tau) {
  return kad::bound_g(btilde, L, omega, tau);
}

kad_status kad_compute_delta(uint32_t n, const uint64_t *count0, uint64_t alpha, uint64_t omega,
                             const double *lambda_l, const double *lambda_u, double delta,
                             double balance_eps, double *L_l, double *L_u, double *C) try {
  if (!n || !count0 || !lambda_l || !lambda_u || !L_l || !L_u || !alpha)
    return fail(KAD_EINVAL, "bad argument");
  if (!(delta > 0 && delta < 1) || !(balance_eps > 0 && balance_eps < 0.5))
    return fail(KAD_EINVAL, "delta must be in (0,1) and balance_eps in (0,0.5)");
  kad::compute_delta(n, count0, alpha, omega, lambda_l, lambda_u, delta, balance_eps, L_l, L_u, C);
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_compute_delta_hist(uint32_t n, const uint64_t *hist, uint64_t cmax, uint64_t alpha,
                                  uint64_t omega, double lambda_l, double lambda_u, double delta,
                                  double balance_eps, uint32_t *group_of_count, double *L_l,
                                  double *L_u, uint32_t *ngroups, double *C) try {
  if (!n || !hist || !alpha || !group_of_count || !L_l || !L_u || !ngroups)
    return fail(KAD_EINVAL, "bad argument");
  if (!(delta > 0 && delta < 1) || !(balance_eps > 0 && balance_eps < 0.5))
    return fail(KAD_EINVAL, "delta must be in (0,1) and balance_eps in (0,0.5)");
  if (cmax >= (1ull << 32)) return fail(KAD_EINVAL, "cmax too large");
  uint64_t total = 0;
  for (uint64_t c = 0; c <= cmax; ++c) total += hist[c];
  if (total != n) return fail(KAD_EINVAL, "the histogram does not count n nodes");
  std::vector<uint32_t> cgrp;
  kad::Groups groups;
  kad::compute_delta_hist(n, hist, cmax, alpha, omega, lambda_l, lambda_u, delta, balance_eps,
                          cgrp, groups, C);
  for (uint64_t c = 0; c <= cmax; ++c) group_of_count[c] = hist[c] ? cgrp[c] : 0u;
  for (size_t g = 0; g < groups.L_l.size(); ++g) {
    L_l[g] = groups.L_l[g];
    L_u[g] = groups.L_u[g];
  }
  *ngroups = (uint32_t)groups.L_l.size();
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_topk_lambdas(uint32_t n, uint32_t k, const uint64_t *count0, uint64_t alpha,
                            double epsilon, double *lambda_l, double *lambda_u) try {
  if (!n || k < 1 || k > n || !count0 || !lambda_l || !lambda_u || !alpha)
    return fail(KAD_EINVAL, "bad argument");
  kad::topk_lambdas(n, k, count0, alpha, epsilon, lambda_l, lambda_u);
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_topk_select(uint32_t n, uint32_t k, const uint64_t *count, const double *lower,
                           const double *upper, uint32_t cap, uint32_t *node, uint32_t *rank_lo,
                           uint32_t *rank_hi, uint32_t *len) try {
  if (!n || k < 1 || k > n || !count || !lower || !upper || !len)
    return fail(KAD_EINVAL, "bad argument");
  std::vector<uint32_t> sel, rlo, rhi;
  kad::topk_select(n, k, count, lower, upper, sel, rlo, rhi);
  *len = (uint32_t)sel.size();
  if (sel.size() > cap) return fail(KAD_ETOOSMALL, "the selection has %zu entries", sel.size());
  for (size_t q = 0; q < sel.size(); ++q) {
    if (node) node[q] = sel[q];
    if (rank_lo) rank_lo[q] = rlo[q];
    if (rank_hi) rank_hi[q] = rhi[q];
  }
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

int kad_have_to_stop(uint32_t n, uint32_t mode, uint32_t k, const uint64_t *count, uint64_t tau,
                     uint64_t omega, double epsilon, const double *L_l, const double *L_u) try {
  if (!n || !count || !L_l || !L_u || tau == 0) return fail(KAD_EINVAL, "bad argument");
  if (mode != KAD_ALL_NODES && mode != KAD_TOPK) return fail(KAD_EINVAL, "bad mode");
  if (mode == KAD_TOPK && (k < 1 || k > n)) return fail(KAD_EINVAL, "k out of range");
  // the same grouped evaluation that kad_run uses at every check
  kad::StopChecker checker(n, mode, k, epsilon, omega, L_l, L_u);
  return checker.check(count, tau) ? 1 : 0;
} catch (...) {
  return kad::status_of_exception();
}

// ---------------------------------------------------------------- sampling primitives

kad_status kad_sample_paths(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                            uint64_t first, uint32_t count, uint32_t *s, uint32_t *t,
                            uint64_t *path_off, uint32_t *path_nodes, uint64_t path_cap,
                            uint64_t *arcs_scanned, uint32_t *flags, void *hip_stream) try {
  if (!ctx || !g) return fail(KAD_EINVAL, "NULL context or graph");
  if (path_nodes && !path_off) return fail(KAD_EINVAL, "path_nodes needs path_off");
  if (phase > 255) return fail(KAD_EINVAL, "phase must fit 8 bits");
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  kad_graph *gm = const_cast<kad_graph *>(g);
  uint32_t vd;
  bool ex;
  kad_status st = graph_vd(gm, &vd, &ex);
  if (st) return st;
  const uint32_t stride = std::max<uint32_t>(vd, 2);
  const int ovc = kad::overflow_class(g, vd, true);
  const uint32_t batch = std::min<uint32_t>(std::max<uint32_t>(count, 1), DEFAULT_BATCH);
  if ((st = ensure_capacity(ctx, g, ovc, batch, stride))) return st;
  hipStream_t stream = pick_stream(ctx, hip_stream);
  HIP_TRY(ctx->h_s.ensure(batch));
  HIP_TRY(ctx->h_t.ensure(batch));
  HIP_TRY(ctx->h_path.ensure((size_t)batch * stride));
  OutSet &o = ctx->outs[0];
  uint64_t off = 0;
  bool short_buf = false;
  for (uint64_t done = 0; done < count;) {
    const uint32_t nb = (uint32_t)std::min<uint64_t>(batch, count - done);
    if ((st = launch_batch(ctx, g, seed, phase, first + done, nb, stride, 0, stream, ovc))) return st;
    HIP_TRY(hipMemcpyAsync(ctx->h_s.p, o.s.p, (size_t)nb * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(ctx->h_t.p, o.t.p, (size_t)nb * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(o.h_len.p, o.len.p, (size_t)nb * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(ctx->h_path.p, o.path.p, (size_t)nb * stride * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if ((st = finish_batch(ctx, 0, nb, 0))) return st;  // flags are reported, not fatal
    for (uint32_t k = 0; k < nb; ++k) {
      const uint64_t idx = done + k;
      if (s) s[idx] = ctx->h_s.p[k];
      if (t) t[idx] = ctx->h_t.p[k];
      if (arcs_scanned) arcs_scanned[idx] = o.h_arcs.p[k];
      if (flags) flags[idx] = o.h_flags.p[k];
      const uint32_t len = o.h_len.p[k];
      if (path_off) path_off[idx] = off;
      if (path_nodes) {
        if (off + len <= path_cap)
          memcpy(path_nodes + off, ctx->h_path.p + (size_t)k * stride, (size_t)len * 4);
        else
          short_buf = true;
      }
      off += len;
    }
    done += nb;
  }
  if (path_off) path_off[count] = off;
  if (short_buf) return fail(KAD_ETOOSMALL, "path_nodes needs %llu entries", (unsigned long long)off);
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_hit_counts(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                          uint64_t first, uint64_t count, uint64_t *count_out,
                          uint64_t *arcs_scanned, void *hip_stream) try {
  if (!ctx || !g || !count_out) return fail(KAD_EINVAL, "NULL argument");
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  kad_graph *gm = const_cast<kad_graph *>(g);
  uint32_t vd;
  bool ex;
  kad_status st = graph_vd(gm, &vd, &ex);
  if (st) return st;
  const uint32_t stride = std::max<uint32_t>(vd, 2);
  const int ovc = kad::overflow_class(g, vd, true);
  const uint32_t batch = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(count, 1), DEFAULT_BATCH);
  if ((st = ensure_capacity(ctx, g, ovc, batch, stride))) return st;
  hipStream_t stream = pick_stream(ctx, hip_stream);
  HIP_TRY(hipMemsetAsync(ctx->count.p, 0, (size_t)g->n * 8, stream));
  uint64_t arcs = 0;
  for (uint64_t done = 0; done < count;) {
    const uint32_t nb = (uint32_t)std::min<uint64_t>(batch, count - done);
    if ((st = launch_batch(ctx, g, seed, phase, first + done, nb, stride, 0, stream, ovc))) return st;
    HIP_TRY(kad::launch_hit_reduce(ctx->outs[0].path.p, ctx->outs[0].len.p, stride, nb, g->n,
                                   ctx->count.p, false, nullptr, nullptr, hit_scratch(ctx), stream));
    if ((st = finish_batch(ctx, 0, nb, nb))) return st;
    for (uint32_t k = 0; k < nb; ++k) arcs += ctx->outs[0].h_arcs.p[k];
    done += nb;
  }
  HIP_TRY(hipMemcpyAsync(ctx->h_count.p, ctx->count.p, (size_t)g->n * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (uint32_t v = 0; v < g->n; ++v) count_out[v] += ctx->h_count.p[v];
  if (arcs_scanned) *arcs_scanned = arcs;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_edge_hit_counts(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                               uint64_t first, uint64_t count, uint64_t *count_out,
                               uint64_t *arcs_scanned, void *hip_stream) try {
  if (!ctx || !g || !count_out) return fail(KAD_EINVAL, "NULL argument");
  if (phase > 255) return fail(KAD_EINVAL, "phase must fit 8 bits");
  const uint64_t items = kad::run_items(g, KAD_TARGET_EDGES);
  if (items == 0) return fail(KAD_EINVAL, "the graph has no edges");
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  kad_graph *gm = const_cast<kad_graph *>(g);
  uint32_t vd;
  bool ex;
  kad_status st = graph_vd(gm, &vd, &ex);
  if (st) return st;
  const uint32_t *edge_ids = nullptr;
  if ((st = kad::graph_edge_ids(gm, &edge_ids))) return st;
  const uint32_t stride = std::max<uint32_t>(vd, 2), rstride = stride + 1;
  const int ovc = kad::overflow_class(g, vd, true);
  const uint32_t batch = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(count, 1), DEFAULT_BATCH);
  if ((st = ensure_capacity(ctx, g, ovc, batch, stride, items, true))) return st;
  hipStream_t stream = pick_stream(ctx, hip_stream);
  HIP_TRY(hipMemsetAsync(ctx->count.p, 0, (size_t)items * 8, stream));
  uint64_t arcs = 0;
  for (uint64_t done = 0; done < count;) {
    const uint32_t nb = (uint32_t)std::min<uint64_t>(batch, count - done);
    if ((st = launch_batch(ctx, g, seed, phase, first + done, nb, stride, 0, stream, ovc, 0,
                           nullptr, nullptr, true, edge_ids)))
      return st;
    HIP_TRY(kad::launch_hit_reduce(ctx->outs[0].epath.p, ctx->outs[0].elen.p, rstride, nb,
                                   (uint32_t)items, ctx->count.p, false, nullptr, nullptr,
                                   hit_scratch(ctx), stream));
    if ((st = finish_batch(ctx, 0, nb, nb))) return st;
    for (uint32_t k = 0; k < nb; ++k) arcs += ctx->outs[0].h_arcs.p[k];
    done += nb;
  }
  HIP_TRY(hipMemcpyAsync(ctx->h_count.p, ctx->count.p, (size_t)items * 8, hipMemcpyDeviceToHost,
                         stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (uint64_t e = 0; e < items; ++e) count_out[e] += ctx->h_count.p[e];
  if (arcs_scanned) *arcs_scanned = arcs;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_graph_edge_count(const kad_graph *g, uint64_t *count) try {
  if (!g || !count) return fail(KAD_EINVAL, "NULL argument");
  *count = kad::run_items(g, KAD_TARGET_EDGES);
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_graph_edge_ids(const kad_graph *g, uint32_t *eid) try {
  if (!g || (!eid && g->arcs)) return fail(KAD_EINVAL, "NULL argument");
  if (g->directed) {
    for (uint64_t e = 0; e < g->arcs; ++e) eid[e] = (uint32_t)e;
    return KAD_OK;
  }
  const uint32_t *d = nullptr;
  kad_status st = kad::graph_edge_ids(const_cast<kad_graph *>(g), &d);
  if (st) return st;
  memcpy(eid, g->eid.data(), (size_t)g->arcs * 4);
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

// ---------------------------------------------------------------- hit counts, no allocation

kad_status kad_hit_counts_noalloc(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                                  uint64_t first, uint64_t count, uint64_t *count_dev,
                                  uint64_t *arcs_dev, uint32_t *flags_dev, void *hip_stream) try {
  if (!ctx || !g || !count_dev || !arcs_dev || !flags_dev) return fail(KAD_EINVAL, "NULL argument");
  if (phase > 255) return fail(KAD_EINVAL, "phase must fit 8 bits");
  if (!ctx->noalloc) return fail(KAD_EDEVICE, "the fixed scratch of this device is not set up");
  if (count == 0) return KAD_OK;
  kad_graph *gm = const_cast<kad_graph *>(g);
  uint32_t vd;
  bool ex;
  kad_status st = graph_vd(gm, &vd, &ex);  // host only, cached on the graph
  if (st) return st;
  if (kad::overflow_class(g, vd, true) != 0)
    return fail(KAD_EINVAL, "path counts of this graph may pass 128 bits: its samples need the "
                "wide-count arena, which the fixed scratch does not hold (use kad_hit_counts)");
  const uint32_t n = g->n, stride = std::max<uint32_t>(vd, 2);
  // layout of the scratch, each region 256-byte aligned: launch counters, per-sample outputs
  // of one launch (C samples), one wide-count slot (arena and level tables), then the
  // sampler slots (node records, reached lists, candidate buffers of PI_SMALL entries)
  constexpr uint32_t PI_SMALL = 4096, MAX_LEV = 1024, C_MAX = 8192;
  const uint64_t total = kad::NOALLOC_SCRATCH_BYTES;
  auto align = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  const uint32_t C = (uint32_t)std::min<uint64_t>(count, C_MAX);
  uint64_t off = 0;
  const uint64_t o_cnt = off;
  off = align(off + 64);
  const uint64_t o_s = off; off = align(off + 4ull * C);
  const uint64_t o_t = off; off = align(off + 4ull * C);
  const uint64_t o_len = off; off = align(off + 4ull * C);
  const uint64_t o_flags = off; off = align(off + 4ull * C);
  const uint64_t o_nodes = off; off = align(off + 4ull * C);
  const uint64_t o_fix = off; off = align(off + 4ull * C);
  const uint64_t o_arcs = off; off = align(off + 8ull * C);
  const uint64_t o_path = off; off = align(off + 4ull * C * stride);
  const uint64_t limbs = 3ull * n + g->arcs + (1ull << 18);
  const uint64_t o_arena = off; off = align(off + 8ull * limbs);
  const uint64_t o_lv = off; off = align(off + 2ull * MAX_LEV * 4 * 4);
  const uint64_t o_lb = off; off = align(off + 2ull * MAX_LEV * 8);
  const uint64_t per_slot = align((uint64_t)n * 4 * kad::REC_WORDS) + align(4ull * n) +
                            8ull * PI_SMALL;
  const kad::LaunchShape shape = kad::graph_shape(g);
  const uint64_t resident = (uint64_t)ctx->cus *
      (uint64_t)ctx->blocks_per_cu[shape.block == 64 ? 0 : (shape.block == 128 ? 1 : 2)];
  const uint64_t room = off < total ? total - off : 0;
  const uint64_t G = std::min<uint64_t>(resident, room / per_slot);
  if (G == 0)
    return fail(KAD_ENOMEM, "graph too large for the fixed scratch of %llu bytes: %llu bytes of "
                "working memory and one sampler slot of %llu bytes are needed",
                (unsigned long long)total, (unsigned long long)off, (unsigned long long)per_slot);
  uint8_t *base = static_cast<uint8_t *>(ctx->noalloc);
  uint32_t *cnt = reinterpret_cast<uint32_t *>(base + o_cnt);
  kad::SampleOut out;
  out.s = reinterpret_cast<uint32_t *>(base + o_s);
  out.t = reinterpret_cast<uint32_t *>(base + o_t);
  out.len = reinterpret_cast<uint32_t *>(base + o_len);
  out.flags = reinterpret_cast<uint32_t *>(base + o_flags);
  out.nodes = reinterpret_cast<uint32_t *>(base + o_nodes);
  out.arcs = reinterpret_cast<uint64_t *>(base + o_arcs);
  out.path = reinterpret_cast<uint32_t *>(base + o_path);
  out.stride = stride;
  out.fix_list = reinterpret_cast<uint32_t *>(base + o_fix);
  out.fix_count = cnt + 1;
  kad::SampleOut wout = out;  // the wide kernel's outputs: it keeps no list
  wout.fix_list = nullptr;
  wout.fix_count = nullptr;
  kad::SlotState sv;
  sv.slots = (uint32_t)G;
  sv.n = n;
  sv.pi_cap = PI_SMALL;
  uint8_t *slots = base + off;
  sv.rec = reinterpret_cast<uint32_t *>(slots);
  sv.visit = reinterpret_cast<uint32_t *>(slots + G * align((uint64_t)n * 4 * kad::REC_WORDS));
  sv.pi = reinterpret_cast<uint64_t *>(slots + G * (align((uint64_t)n * 4 * kad::REC_WORDS) +
                                                    align(4ull * n)));
  kad::WideState wv;  // one wide-count slot, on sampler slot 0's node records
  wv.slots = 1;
  wv.max_lev = MAX_LEV;
  wv.arena_limbs = limbs;
  wv.arena = reinterpret_cast<uint64_t *>(base + o_arena);
  wv.lv = reinterpret_cast<uint32_t *>(base + o_lv);
  wv.lbase = reinterpret_cast<uint64_t *>(base + o_lb);
  // NULL is the device's null stream: the work is only enqueued, so the caller must be able
  // to order its own work after it
  hipStream_t stream = (hipStream_t)hip_stream;
  HIP_TRY(hipSetDevice(ctx->device));
  // node records start all zero (the kernels leave them so, but the region may have held
  // other data in an earlier call with another layout); cleared by a kernel, not a memset
  HIP_TRY(kad::launch_zero_u32(sv.rec, (uint64_t)G * n * kad::REC_WORDS, stream));
  const kad::GraphDev gd = dev_view(g);
  for (uint64_t done = 0; done < count;) {
    const uint32_t nb = (uint32_t)std::min<uint64_t>(C, count - done);
    HIP_TRY(kad::launch_zero_u32(cnt, 3, stream));
    HIP_TRY(kad::launch_sampler(gd, sv, seed, phase, first + done, nb, cnt, out,
                                (uint32_t)std::min<uint64_t>(G, nb), shape, stream));
    HIP_TRY(kad::launch_wide_fix(gd, seed, phase, first + done, nullptr, 0, sv, wv, nb, false,
                                 out.fix_list, cnt + 1, cnt + 2, wout, stream));
    HIP_TRY(kad::launch_hit_add_atomic(out.path, out.len, stride, nb, n, count_dev, stream));
    HIP_TRY(kad::launch_sample_sums(out.arcs, out.flags, nb, arcs_dev, flags_dev, stream));
    done += nb;
  }
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

// ---------------------------------------------------------------- the adaptive run

kad_status kad_run(kad_ctx *ctx, const kad_graph *g, const kad_params *p, kad_result *r,
                   void *hip_stream) try {
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  if (!ctx || !g || !p || !r) return fail(KAD_EINVAL, "NULL argument");
  kad_status st = kad::validate_params(g, p);
  if (st) return st;
  const double c = p->c > 0 ? p->c : 0.5;
  const double eb = p->balance_eps > 0 ? p->balance_eps : 0.001;
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  kad_graph *gm = const_cast<kad_graph *>(g);
  // the run's items -- the nodes, or the edges -- and every per-item array and counter below
  const bool edges = p->target == KAD_TARGET_EDGES;
  const uint32_t n = (uint32_t)kad::run_items(g, p->target);
  const uint32_t *edge_ids = nullptr;
  if (edges && (st = kad::graph_edge_ids(gm, &edge_ids))) return st;
  ctx->run_wide = 0;

  uint32_t vd;
  bool vd_exact = false;
  if (p->vd_override) {
    vd = p->vd_override;
  } else if ((st = graph_vd(gm, &vd, &vd_exact))) {
    return st;
  }
  const uint64_t omega = edges ? kad::omega_edges_of(p->epsilon, p->delta, vd, c)
                               : kad::omega_of(p->epsilon, p->delta, vd, c);
  const uint64_t alpha = kad::alpha_of(omega);
  const uint64_t B = p->check_interval ? p->check_interval : kad::interval_of(omega);
  uint64_t K = p->kernel_batch ? p->kernel_batch : DEFAULT_BATCH;
  K = std::max<uint64_t>(B, (K + B - 1) / B * B);
  if (K > (1u << 30)) return fail(KAD_EINVAL, "kernel_batch too large");
  const uint32_t chunks_per_batch = (uint32_t)(K / B);
  const uint32_t stride = std::max<uint32_t>(vd, 2);
  const int ovc = kad::overflow_class(g, vd, p->vd_override == 0);
  if ((st = ensure_capacity(ctx, g, ovc, (uint32_t)K, stride, n, edges))) return st;
  // what the hit reductions read: the node paths, or the same paths as edge ids
  const uint32_t rstride = edges ? stride + 1 : stride;
  auto rpath = [&](const OutSet &o) -> const uint32_t * { return edges ? o.epath.p : o.path.p; };
  auto rlen = [&](const OutSet &o) -> const uint32_t * { return edges ? o.elen.p : o.len.p; };
  hipStream_t stream = pick_stream(ctx, hip_stream);
  // main-phase batches as recorded chains (not while timing: its events sit between the
  // launches), or the plain single-graph path
  const bool graph_mode = ctx->exec == KAD_EXEC_GRAPH && !ctx->timing;
  const bool plain = ctx->exec == KAD_EXEC_PLAIN;
  const uint32_t plain_grid = kad::launch_grid(ctx, kad::graph_shape(g), UINT32_MAX);
  if ((st = run_timing_begin(ctx, stream))) return st;
  struct RunTimingEnd {  // also on early returns
    kad_ctx *c;
    ~RunTimingEnd() { run_timing_end(c); }
  } run_timing_guard{ctx};
  const auto t_setup = clock::now();

  if (p->schedule != KAD_SCHEDULE_ADAPTIVE) {
    // ---- a fixed number of main-phase samples, no pilot and no stopping check
    const uint64_t tau_fixed =
        edges && p->schedule == KAD_SCHEDULE_RK
            ? kad::omega_edges_of(p->epsilon, 2.0 * p->delta, vd, c)  // ln(1/delta): 2 delta
            : kad_fixed_samples(p->schedule, p->epsilon, p->delta, vd, n, c);
    HIP_TRY(hipMemsetAsync(ctx->count.p, 0, (size_t)n * 8, stream));
    uint64_t arcs_f = 0;
    for (uint64_t done = 0; done < tau_fixed;) {
      const uint32_t nb = (uint32_t)std::min<uint64_t>(ctx->outs[0].cap, tau_fixed - done);
      if ((st = launch_batch(ctx, g, p->seed, 1, done, nb, stride, 0, stream, ovc, 0, nullptr,
                             nullptr, edges, edge_ids)))
        return st;
      HIP_TRY(kad::launch_hit_reduce(rpath(ctx->outs[0]), rlen(ctx->outs[0]), rstride, nb, n,
                                     ctx->count.p, false, nullptr, nullptr, hit_scratch(ctx), stream));
      if ((st = finish_batch(ctx, 0, nb, nb))) return st;
      for (uint32_t k = 0; k < nb; ++k) arcs_f += ctx->outs[0].h_arcs.p[k];
      done += nb;
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_count.p, ctx->count.p, (size_t)n * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    run_timing_end(ctx);
    const auto t_main_f = clock::now();
    r->tau = tau_fixed;
    r->omega = tau_fixed;
    r->alpha = 0;
    r->interval = 0;
    r->arcs_scanned = arcs_f;
    r->pilot_arcs_scanned = 0;
    r->overflow_samples = ctx->run_wide;
    r->vd = vd;
    r->vd_exact = vd_exact ? 1u : 0u;
    r->stop_reason = KAD_STOP_FIXED;
    r->n = g->n;
    r->items = n;
    r->C = 0.0;
    const uint64_t *cnt = ctx->h_count.p;
    std::vector<double> &bcs = ctx->h_bc, &los = ctx->h_lo, &his = ctx->h_hi;
    double *bc = r->bc ? r->bc : (bcs.resize(n), bcs.data());
    double *lo = r->lower ? r->lower : (los.resize(n), los.data());
    double *hi = r->upper ? r->upper : (his.resize(n), his.data());
    if (r->count) memcpy(r->count, cnt, (size_t)n * 8);
    kad::node_outputs(n, cnt, tau_fixed, tau_fixed, false, p->epsilon, nullptr, nullptr, {}, bc,
                      lo, hi);
    r->topk_len = 0;
    kad_status ret = KAD_OK;
    if (p->mode == KAD_TOPK) {
      std::vector<uint32_t> sel, rlo, rhi;
      kad::topk_select(n, p->k, cnt, lo, hi, sel, rlo, rhi);
      r->topk_len = (uint32_t)sel.size();
      if (sel.size() > r->topk_cap) {
        ret = fail(KAD_ETOOSMALL, "top-k output needs %zu entries", sel.size());
      } else {
        for (size_t q = 0; q < sel.size(); ++q) {
          if (r->topk_node) r->topk_node[q] = sel[q];
          if (r->rank_lo) r->rank_lo[q] = rlo[q];
          if (r->rank_hi) r->rank_hi[q] = rhi[q];
        }
      }
    }
    const auto t_end_f = clock::now();
    auto secs_f = [](clock::time_point a, clock::time_point b) {
      return std::chrono::duration<double>(b - a).count();
    };
    r->seconds = secs_f(t0, t_end_f);
    r->seconds_setup = secs_f(t0, t_setup);
    r->seconds_pilot = 0.0;
    r->seconds_delta = 0.0;
    r->seconds_main = secs_f(t_setup, t_main_f);
    return ret;
  }

  // ---- pilot (phase 0): alpha samples -> count0
  std::vector<uint64_t> &count0 = ctx->h_count0;
  // All-nodes runs have the same half-width at every node, so computeDelta needs only
  // the histogram of the pilot counts (at most alpha + 1 bins): the counts stay on the
  // device, and the node -> group map is built there too.
  const bool pilot_hist = p->mode == KAD_ALL_NODES && alpha < (1u << 24);
  const uint32_t bins = pilot_hist ? (uint32_t)alpha + 1 : 0u;
  if (pilot_hist) {
    HIP_TRY(ctx->count0d.ensure(n));
    HIP_TRY(ctx->hist.ensure(bins));
    HIP_TRY(ctx->cgrp.ensure(bins));
    HIP_TRY(ctx->h_hist.ensure(bins));
    HIP_TRY(ctx->h_cgrp.ensure(bins));
    HIP_TRY(ctx->h_count0p.ensure(n));
  } else {
    count0.resize(n);
  }
  uint64_t *pcount = pilot_hist ? ctx->count0d.p : ctx->count.p;
  HIP_TRY(hipMemsetAsync(pcount, 0, (size_t)n * 8, stream));
  // The first main-phase batch (phase 1 does not depend on the pilot): half the cap, in
  // whole check intervals.  When the slots allow it, it runs beside the pilot on its own
  // stream, slots and work counter (a pilot of alpha samples is one short launch whose
  // last samples would otherwise hold the GPU); its wide-count fix, which shares one
  // arena, waits for the pilot's.  Its slots start past every slot the pilot may use:
  // the pilot sampler's (at most alpha) and, when the wide-count kernel shares the
  // sampler slots (one record per node), those of the pilot's wide-count passes, which
  // run on sampler slots 0, 1, ... (at most w_slots).
  const int first_set = 1;
  const uint32_t first_nb = (uint32_t)std::min<uint64_t>(
      omega, std::min<uint64_t>(K, std::max<uint64_t>(B, (omega / 2 + B - 1) / B * B)));
  const uint32_t b1_slot0 = (uint32_t)std::max<uint64_t>(
      std::max<uint64_t>(alpha, 64), ctx->slot_hbits ? 0u : ctx->w_slots);
  const bool overlap = !plain && hip_stream == nullptr && ovc != 2 && alpha <= ctx->outs[0].cap &&
                       (uint64_t)ctx->slots >= (uint64_t)b1_slot0 + kad::launch_grid(
                                                   ctx, kad::graph_shape(g), first_nb);
  hipStream_t b1_stream = overlap ? ctx->pstream : stream;
  uint64_t pilot_arcs = 0;
  uint32_t pilot_last = 0;
  for (uint64_t done = 0; done < alpha;) {
    if (pilot_last) {  // several pilot batches: the previous one must be read first
      if ((st = finish_batch(ctx, 0, pilot_last, pilot_last))) return st;
      for (uint32_t k = 0; k < pilot_last; ++k) pilot_arcs += ctx->outs[0].h_arcs.p[k];
    }
    // (the plain path: at most one resident grid, one sample per workgroup)
    const uint32_t nb = (uint32_t)std::min<uint64_t>(
        std::min<uint64_t>(ctx->outs[0].cap, plain ? plain_grid : UINT32_MAX), alpha - done);
    if ((st = launch_batch(ctx, g, p->seed, 0, done, nb, stride, 0, stream, ovc, 0, nullptr,
                           nullptr, edges, edge_ids)))
      return st;
    if (overlap) {
      HIP_TRY(hipStreamWaitEvent(b1_stream, ctx->outs[first_set].reduced, 0));
      if ((st = launch_batch(ctx, g, p->seed, 1, 0, first_nb, stride, first_set, b1_stream, ovc,
                             b1_slot0, ctx->work2.p, ctx->outs[0].copied, edges, edge_ids)))
        return st;
    }
    HIP_TRY(kad::launch_hit_reduce(rpath(ctx->outs[0]), rlen(ctx->outs[0]), rstride, nb, n,
                                   pcount, false, nullptr, nullptr, hit_scratch(ctx), stream));
    pilot_last = nb;
    done += nb;
  }
  if (pilot_hist) {
    HIP_TRY(kad::launch_zero_u32(ctx->hist.p, bins, stream));
    HIP_TRY(kad::launch_count_hist(ctx->count0d.p, n, ctx->hist.p, bins, stream));
    HIP_TRY(hipMemcpyAsync(ctx->h_hist.p, ctx->hist.p, (size_t)bins * 4, hipMemcpyDeviceToHost,
                           stream));
  } else {
    HIP_TRY(hipMemcpyAsync(count0.data(), ctx->count.p, (size_t)n * 8, hipMemcpyDeviceToHost,
                           stream));
  }
  hipEvent_t pilot_done = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&pilot_done, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(pilot_done, stream));

  // ---- otherwise the first main-phase batch follows the pilot on the stream and is
  // sampled while the host runs computeDelta
  if (!overlap && !plain) {
    HIP_TRY(hipStreamWaitEvent(stream, ctx->outs[first_set].reduced, 0));
    st = graph_mode ? replay_sampling(ctx, g, first_set, p->seed, 1, 0, first_nb, (uint32_t)K,
                                      stride, stream, ovc, edges, edge_ids)
                    : launch_batch(ctx, g, p->seed, 1, 0, first_nb, stride, first_set, stream,
                                   ovc, 0, nullptr, nullptr, edges, edge_ids);
    if (st) {
      (void)hipEventDestroy(pilot_done);
      return st;
    }
  }
  HIP_TRY(wait_event(pilot_done));
  (void)hipEventDestroy(pilot_done);
  if ((st = finish_batch(ctx, 0, pilot_last, pilot_last))) return st;
  for (uint32_t k = 0; k < pilot_last; ++k) pilot_arcs += ctx->outs[0].h_arcs.p[k];
  const auto t_pilot = clock::now();

  // ---- computeDelta (host, binary64)
  std::vector<double> &lam_l = ctx->h_lam_l, &lam_u = ctx->h_lam_u, &L_l = ctx->h_L_l,
                      &L_u = ctx->h_L_u;
  double Cb = 0;
  kad::Groups groups;
  std::vector<uint32_t> cgrp_h;   // pilot_hist: pilot count -> group
  std::vector<double> gLl, gLu;   // pilot_hist: group -> L values
  if (pilot_hist) {
    std::vector<uint64_t> h64(bins);
    for (uint32_t c = 0; c < bins; ++c) h64[c] = ctx->h_hist.p[c];
    kad::compute_delta_hist(n, h64.data(), bins - 1, alpha, omega, p->epsilon, p->epsilon,
                            p->delta, eb, cgrp_h, groups, &Cb);
    gLl = groups.L_l;
    gLu = groups.L_u;
  } else {
    lam_l.assign(n, p->epsilon);
    lam_u.assign(n, p->epsilon);
    L_l.resize(n);
    L_u.resize(n);
    if (p->mode == KAD_TOPK) kad::topk_lambdas(n, p->k, count0.data(), alpha, p->epsilon, lam_l.data(), lam_u.data());
    kad::compute_delta(n, count0.data(), alpha, omega, lam_l.data(), lam_u.data(), p->delta, eb,
                       L_l.data(), L_u.data(), &Cb, &groups);
  }
  // (per-node L arrays are read only by the top-k check, never on the histogram path)
  kad::StopChecker checker(n, p->mode, p->k, p->epsilon, omega,
                           pilot_hist ? nullptr : L_l.data(), pilot_hist ? nullptr : L_u.data(),
                           std::move(groups));

  const auto t_delta = clock::now();

  // ---- main phase (phase 1): batches of samples, a check every B samples.
  // The sampler runs on `stream`; the hit reductions and the check snapshots on the
  // context's reduction stream.  Batch b+1 is launched once every check of batch b is
  // made, sized from how far its last check is from stopping (launched earlier, its grid
  // holds every CU while batch b's reductions wait); batch sizes never change the result,
  // because the check is made at every multiple of B whatever the batches are.
  // All-nodes: the reduction also keeps each stopping group's largest count on the
  // device, so a check copies only those maxima.  Top-k: a check copies the counts.
  hipStream_t rs = ctx->rstream;
  const bool by_group = p->mode == KAD_ALL_NODES;
  const size_t ngroups = checker.groups();
  const size_t snap = by_group ? ngroups : (size_t)n;
  HIP_TRY(hipMemsetAsync(ctx->count.p, 0, (size_t)n * 8, rs));
  if (by_group) {
    HIP_TRY(ctx->group.ensure(n));
    HIP_TRY(ctx->gmax.ensure(ngroups));
    if (pilot_hist) {
      memcpy(ctx->h_cgrp.p, cgrp_h.data(), (size_t)bins * 4);
      HIP_TRY(hipMemcpyAsync(ctx->cgrp.p, ctx->h_cgrp.p, (size_t)bins * 4, hipMemcpyHostToDevice,
                             rs));
      HIP_TRY(kad::launch_group_map(ctx->count0d.p, n, ctx->cgrp.p, bins, ctx->group.p, rs));
      // the pilot counts, for the intervals at the end (off the critical path)
      HIP_TRY(hipMemcpyAsync(ctx->h_count0p.p, ctx->count0d.p, (size_t)n * 8,
                             hipMemcpyDeviceToHost, rs));
    } else {
      HIP_TRY(hipMemcpyAsync(ctx->group.p, checker.group_of().data(), (size_t)n * 4,
                             hipMemcpyHostToDevice, rs));
    }
    HIP_TRY(hipMemsetAsync(ctx->gmax.p, 0, ngroups * 8, rs));
  }
  PinBuf<uint64_t> &snaps = ctx->snaps;  // one snapshot per check of the current batch
  HIP_TRY(snaps.ensure(snap * chunks_per_batch));
  // All-nodes runs reduce a batch's check intervals together (launch_hit_batch) when the
  // per-interval hit counters fit 256 MiB; its scratch is cleared here, beside the pilot.
  const bool batch_reduce = by_group && chunks_per_batch >= 2 &&
                            (uint64_t)n * chunks_per_batch * 4 <= (256ull << 20);
  if (batch_reduce) {
    HIP_TRY(ctx->ivtmp.ensure((size_t)n * chunks_per_batch));
    HIP_TRY(ctx->ivmax.ensure((size_t)chunks_per_batch * ngroups));
    HIP_TRY(kad::launch_zero_u32(ctx->ivtmp.p, (uint64_t)n * chunks_per_batch, rs));
    HIP_TRY(kad::launch_zero_u32(reinterpret_cast<uint32_t *>(ctx->ivmax.p),
                                 (uint64_t)chunks_per_batch * ngroups * 2, rs));
  }
  while (ctx->chunk_ev.size() < chunks_per_batch) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->chunk_ev.push_back(e);
  }
  auto round_up = [&](double x) {
    const double q = std::ceil(std::max(x, 1.0) / (double)B);
    return (uint64_t)std::min<double>(q, (double)(K / B)) * B;
  };

  // The final counts come back in parts, each with its event, so that the host's pass
  // over the nodes (after the loop) starts on the first part while the others are in
  // flight; they are enqueued as soon as the stopping point is known.
  constexpr uint32_t OUT_PARTS = 4;
  while (ctx->chunk_ev.size() < OUT_PARTS) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->chunk_ev.push_back(e);
  }
  uint32_t part_lo[OUT_PARTS + 1];
  for (uint32_t q = 0; q <= OUT_PARTS; ++q) part_lo[q] = (uint32_t)((uint64_t)n * q / OUT_PARTS);
  auto enqueue_count_copy = [&]() -> kad_status {
    for (uint32_t q = 0; q < OUT_PARTS; ++q) {
      if (part_lo[q + 1] > part_lo[q])
        HIP_TRY(hipMemcpyAsync(ctx->h_count.p + part_lo[q], ctx->count.p + part_lo[q],
                               (size_t)(part_lo[q + 1] - part_lo[q]) * 8, hipMemcpyDeviceToHost,
                               rs));
      HIP_TRY(hipEventRecord(ctx->chunk_ev[q], rs));
    }
    return KAD_OK;
  };

  uint64_t tau = 0, arcs = 0, launched = first_nb;
  bool rule = false, stop = false;
  int cur = first_set;
  uint32_t cur_nb = first_nb;
  double worst = 0.0;
  if (plain) {
    // the plain path: every check interval sampled by launches of at most one resident
    // grid (one sample per workgroup), reduced, copied and checked before the next
    HIP_TRY(wait_stream(ctx, rs));  // counters, groups and maxima set up
    const OutSet &o = ctx->outs[0];
    while (!stop) {
      const uint32_t cb = (uint32_t)std::min<uint64_t>(B, omega - tau);
      for (uint32_t d = 0; d < cb;) {
        const uint32_t nb = std::min(plain_grid, cb - d);
        if ((st = launch_batch(ctx, g, p->seed, 1, tau + d, nb, stride, 0, stream, ovc, 0,
                               nullptr, nullptr, edges, edge_ids)))
          return st;
        HIP_TRY(kad::launch_hit_reduce(rpath(o), rlen(o), rstride, nb, n, ctx->count.p, false,
                                       by_group ? ctx->group.p : nullptr,
                                       by_group ? ctx->gmax.p : nullptr, hit_scratch(ctx),
                                       stream));
        if ((st = finish_batch(ctx, 0, nb, nb))) return st;
        for (uint32_t k = 0; k < nb; ++k) arcs += o.h_arcs.p[k];
        d += nb;
      }
      HIP_TRY(hipMemcpyAsync(snaps.p, by_group ? ctx->gmax.p : ctx->count.p, snap * 8,
                             hipMemcpyDeviceToHost, stream));
      HIP_TRY(wait_stream(ctx, stream));
      tau += cb;
      if (tau >= omega) {
        stop = true;
      } else if (cb == B && (by_group ? checker.check_group_max(snaps.p, tau, &worst)
                                      : checker.check(snaps.p, tau))) {
        stop = true;
        rule = true;
      }
    }
    if ((st = enqueue_count_copy())) return st;
  }
  while (!stop) {
    if (cur_nb == 0) return fail(KAD_EINVAL, "internal: empty batch before the stopping point");
    const OutSet &o = ctx->outs[cur];
    HIP_TRY(hipStreamWaitEvent(rs, o.sampled, 0));
    const uint32_t nch = (uint32_t)((cur_nb + B - 1) / B);
    uint32_t queued = 0;  // check intervals whose reduction and snapshot are enqueued
    auto enqueue_upto = [&](uint32_t upto) -> kad_status {
      for (; queued < upto; ++queued) {
        const uint32_t q0 = queued * (uint32_t)B;
        const uint32_t cb = (uint32_t)std::min<uint64_t>(B, cur_nb - q0);
        HIP_TRY(kad::launch_hit_reduce(rpath(o) + (size_t)q0 * rstride, rlen(o) + q0, rstride, cb, n,
                                       ctx->count.p, false, by_group ? ctx->group.p : nullptr,
                                       by_group ? ctx->gmax.p : nullptr, hit_scratch(ctx), rs));
        HIP_TRY(hipMemcpyAsync(snaps.p + (size_t)queued * snap,
                               by_group ? ctx->gmax.p : ctx->count.p, snap * 8,
                               hipMemcpyDeviceToHost, rs));
        HIP_TRY(hipEventRecord(ctx->chunk_ev[queued], rs));
        if (queued + 1 == nch) HIP_TRY(hipEventRecord(ctx->outs[cur].reduced, rs));
      }
      return KAD_OK;
    };
    if (batch_reduce) {  // every interval in three launches; all snapshots land together
      if (graph_mode) {
        if ((st = replay_reduce(ctx, cur, rpath(o), rlen(o), rstride, cur_nb, (uint32_t)K,
                                (uint32_t)B, n, (uint32_t)ngroups, snaps.p, rs)))
          return st;
      } else {
        HIP_TRY(kad::launch_hit_batch(rpath(o), rlen(o), rstride, cur_nb, (uint32_t)B, n,
                                      ctx->count.p, ctx->group.p, ctx->gmax.p,
                                      (uint32_t)ngroups, ctx->ivtmp.p, ctx->ivmax.p, snaps.p,
                                      rs));
      }
      for (uint32_t q = 0; q < nch; ++q) HIP_TRY(hipEventRecord(ctx->chunk_ev[q], rs));
      HIP_TRY(hipEventRecord(ctx->outs[cur].reduced, rs));
      queued = nch;
    } else if ((st = enqueue_upto(nch))) {  // every interval, before the next batch
      return st;
    }
    uint32_t next_nb = 0;
    auto launch_next = [&]() -> kad_status {
      if (launched >= omega) return KAD_OK;
      // remaining samples predicted from the last check (the bounds shrink about as
      // 1/tau), but at most half of what has been launched: a prediction made at an early
      // check is coarse, and a later batch is sized from a later check
      double want = (double)K;
      if (by_group && worst > 0.0 && tau > 0) want = (double)tau * worst - (double)launched;
      want = std::min(want, 0.5 * (double)launched);
      next_nb = (uint32_t)std::min<uint64_t>(round_up(want), omega - launched);
      const int nxt = 1 - cur;
      HIP_TRY(hipStreamWaitEvent(stream, ctx->outs[nxt].reduced, 0));
      kad_status s2 =
          graph_mode ? replay_sampling(ctx, g, nxt, p->seed, 1, launched, next_nb, (uint32_t)K,
                                       stride, stream, ovc, edges, edge_ids)
                     : launch_batch(ctx, g, p->seed, 1, launched, next_nb, stride, nxt, stream,
                                    ovc, 0, nullptr, nullptr, edges, edge_ids);
      if (s2) return s2;
      launched += next_nb;
      return KAD_OK;
    };
    uint32_t c = 0, c0 = 0;
    for (; c0 < cur_nb; ++c, c0 += (uint32_t)B) {
      const uint32_t cb = (uint32_t)std::min<uint64_t>(B, cur_nb - c0);
      HIP_TRY(wait_event(ctx->chunk_ev[c]));
      tau += cb;
      const uint64_t *sp = snaps.p + (size_t)c * snap;
      if (tau >= omega) {
        stop = true;
      } else if (cb == B && (by_group ? checker.check_group_max(sp, tau, &worst)
                                      : checker.check(sp, tau))) {
        stop = true;
        rule = true;
      }
      if (stop) break;
    }
    const uint32_t used = stop ? c0 + (uint32_t)std::min<uint64_t>(B, cur_nb - c0) : cur_nb;
    // the GPU's next work first, then this batch's host accounting (its flags and arcs)
    if (stop) {
      // undo the reductions enqueued past the stopping point; the counts go home
      const uint32_t reduced_end = (uint32_t)std::min<uint64_t>((uint64_t)queued * B, cur_nb);
      if (used < reduced_end)
        HIP_TRY(kad::launch_hit_reduce(rpath(o) + (size_t)used * rstride, rlen(o) + used, rstride,
                                       reduced_end - used, n, ctx->count.p, true, nullptr, nullptr,
                                       hit_scratch(ctx), rs));
      if ((st = enqueue_count_copy())) return st;
    } else {
      // the next batch, sized from this batch's last check: its reductions ran on an
      // idle GPU (beside a sampler grid they wait for its last workgroups)
      if ((st = launch_next())) return st;
    }
    if ((st = finish_batch(ctx, cur, cur_nb, used))) return st;
    for (uint32_t k = 0; k < used; ++k) arcs += ctx->outs[cur].h_arcs.p[k];
    if (stop) break;
    cur = 1 - cur;
    cur_nb = next_nb;
  }
  HIP_TRY(wait_stream(ctx, stream));
  if (overlap) HIP_TRY(wait_stream(ctx, b1_stream));
  run_timing_end(ctx);
  const auto t_main = clock::now();

  // ---- outputs (Theorem 1 intervals)
  r->tau = tau;
  r->omega = omega;
  r->alpha = alpha;
  r->interval = B;
  r->arcs_scanned = arcs;
  r->pilot_arcs_scanned = pilot_arcs;
  r->overflow_samples = ctx->run_wide;
  r->vd = vd;
  r->vd_exact = vd_exact ? 1u : 0u;
  r->stop_reason = rule ? KAD_STOP_RULE : KAD_STOP_OMEGA;
  r->n = g->n;
  r->items = n;
  r->C = Cb;
  const uint64_t *cnt = ctx->h_count.p;
  // per-node outputs, written straight into the caller's arrays when given
  std::vector<double> &bcs = ctx->h_bc, &los = ctx->h_lo, &his = ctx->h_hi;
  const bool topk = p->mode == KAD_TOPK;
  double *bc = r->bc ? r->bc : (bcs.resize(n), bcs.data());
  double *lo = r->lower && !topk ? r->lower : (los.resize(n), los.data());
  double *hi = r->upper && !topk ? r->upper : (his.resize(n), his.data());
  if (pilot_hist) {
    // one pass; each worker first waits for the parts that hold its range
    std::atomic<int> werr{0};
    kad::node_outputs_pilot(n, cnt, tau, omega, rule, p->epsilon, ctx->h_count0p.p, cgrp_h, gLl,
                            gLu, bc, lo, hi, r->count, [&](uint32_t ve) {
                              for (uint32_t q = 0; q < OUT_PARTS && part_lo[q] < ve; ++q)
                                if (wait_event(ctx->chunk_ev[q]) != hipSuccess) werr = 1;
                            });
    HIP_TRY(wait_event(ctx->chunk_ev[OUT_PARTS - 1]));
    if (werr) return fail(KAD_EDEVICE, "copying the counts back failed");
  } else {
    HIP_TRY(wait_event(ctx->chunk_ev[OUT_PARTS - 1]));
    if (r->count)
      kad::parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned) {
        memcpy(r->count + vb, cnt + vb, (size_t)(ve - vb) * 8);
      });
    kad::node_outputs(n, cnt, tau, omega, rule, p->epsilon, L_l.data(), L_u.data(),
                      checker.group_of(), bc, lo, hi);
  }
  if (topk) {
    if (r->lower) memcpy(r->lower, lo, (size_t)n * 8);
    if (r->upper) memcpy(r->upper, hi, (size_t)n * 8);
  }
  r->topk_len = 0;
  kad_status ret = KAD_OK;
  if (topk) {
    std::vector<uint32_t> sel, rlo, rhi;
    kad::topk_select(n, p->k, cnt, lo, hi, sel, rlo, rhi);
    r->topk_len = (uint32_t)sel.size();
    if (sel.size() > r->topk_cap) {
      ret = fail(KAD_ETOOSMALL, "top-k output needs %zu entries", sel.size());
    } else {
      for (size_t q = 0; q < sel.size(); ++q) {
        if (r->topk_node) r->topk_node[q] = sel[q];
        if (r->rank_lo) r->rank_lo[q] = rlo[q];
        if (r->rank_hi) r->rank_hi[q] = rhi[q];
      }
    }
  }
  const auto t_end = clock::now();
  auto secs = [](clock::time_point a, clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
  };
  r->seconds = secs(t0, t_end);
  r->seconds_setup = secs(t0, t_setup);
  r->seconds_pilot = secs(t_setup, t_pilot);
  r->seconds_delta = secs(t_pilot, t_delta);
  r->seconds_main = secs(t_delta, t_main);
  return ret;
} catch (...) {
  return kad::status_of_exception();
}

// ---------------------------------------------------------------- launch shape

kad_status kad_graph_set_launch(kad_graph *g, uint32_t block, uint32_t small_expansion) try {
  if (!g) return fail(KAD_EINVAL, "NULL graph");
  if (block == 0 && small_expansion == 0) {
    g->shape_set = false;
    g->shape = kad::LaunchShape{};
    return KAD_OK;
  }
  if (block != 64 && block != 128 && block != 256)
    return fail(KAD_EINVAL, "block must be 64, 128 or 256");
  g->shape.block = (int)block;
  g->shape.small_exp = small_expansion;
  g->shape_set = true;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_graph_set_search(kad_graph *g, uint32_t search) try {
  if (!g) return fail(KAD_EINVAL, "NULL graph");
  if (search != KAD_SEARCH_BALANCED && search != KAD_SEARCH_FORWARD)
    return fail(KAD_EINVAL, "search must be KAD_SEARCH_BALANCED or KAD_SEARCH_FORWARD");
  g->search = search;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_graph_get_search(const kad_graph *g, uint32_t *search) try {
  if (!g || !search) return fail(KAD_EINVAL, "NULL argument");
  *search = g->search;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_graph_get_launch(const kad_graph *g, uint32_t *block, uint32_t *small_expansion) try {
  if (!g) return fail(KAD_EINVAL, "NULL graph");
  const kad::LaunchShape sh = kad::graph_shape(g);
  if (block) *block = (uint32_t)sh.block;
  if (small_expansion) *small_expansion = sh.small_exp;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_autotune(kad_ctx *ctx, kad_graph *g, uint32_t samples, uint32_t *block,
                        uint32_t *small_expansion, double *seconds) try {
  if (!ctx || !g) return fail(KAD_EINVAL, "NULL argument");
  if (samples == 0) samples = DEFAULT_BATCH;
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  uint32_t vd;
  bool ex;
  kad_status st = graph_vd(g, &vd, &ex);
  if (st) return st;
  const uint32_t stride = std::max<uint32_t>(vd, 2);
  const int ovc = kad::overflow_class(g, vd, true);
  if ((st = ensure_capacity(ctx, g, ovc, samples, stride))) return st;
  const kad::LaunchShape saved = g->shape;
  const bool saved_set = g->shape_set;
  const uint32_t exps[4] = {0, 32, 128, 512};
  kad::LaunchShape best;
  double best_s = 1e300;
  auto time_shape = [&](double *t_min) -> kad_status {
    *t_min = 1e300;
    for (int rep = 0; rep < 2; ++rep) {  // the faster of two launches
      kad_status s2 = launch_batch(ctx, g, 1, 1, 0, samples, stride, 0, ctx->stream, ovc);
      if (s2) return s2;
      HIP_TRY(hipStreamSynchronize(ctx->stream));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->outs[0].k0, ctx->outs[0].k1));
      *t_min = std::min(*t_min, ms * 1e-3);
    }
    return KAD_OK;
  };
  g->shape_set = true;
  for (int b : kad::SAMPLER_BLOCKS)
    for (uint32_t e : exps) {
      g->shape.block = b;
      g->shape.small_exp = e;
      double t = 0;
      if ((st = time_shape(&t))) {
        g->shape = saved;
        g->shape_set = saved_set;
        return st;
      }
      if (t < best_s) {
        best_s = t;
        best = g->shape;
      }
    }
  g->shape = best;
  if (block) *block = (uint32_t)best.block;
  if (small_expansion) *small_expansion = best.small_exp;
  if (seconds) *seconds = best_s;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

// ---------------------------------------------------------------- timing (bench support)

kad_status kad_ctx_set_timing(kad_ctx *ctx, int enable) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  ctx->timing = enable != 0;
  ctx->t_launches = ctx->t_samples = ctx->t_arcs = ctx->t_nodes = ctx->t_hits = 0;
  ctx->t_seconds = 0.0;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_set_wide(kad_ctx *ctx, uint32_t slots, uint64_t limbs) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  if (limbs != 0 && limbs < 4096) return fail(KAD_EINVAL, "a wide-count arena needs 4096 limbs or more");
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipDeviceSynchronize());  // no launch may still use the arena
  ctx->w_user_slots = slots;
  ctx->w_user_limbs = limbs;
  ctx->w_arena.release();  // laid out again on next use
  ctx->w_lv.release();
  ctx->w_lbase.release();
  ctx->w_slots = ctx->w_slots2 = 0;
  ctx->w_arena_limbs = ctx->w_arena_limbs2 = 0;
  ctx->w_big = false;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_get_wide(kad_ctx *ctx, uint32_t *slots, uint64_t *limbs, uint32_t *slots2,
                            uint64_t *limbs2) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  if (slots) *slots = ctx->w_slots;
  if (limbs) *limbs = ctx->w_arena_limbs;
  if (slots2) *slots2 = ctx->w_slots2;
  if (limbs2) *limbs2 = ctx->w_arena_limbs2;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_set_table(kad_ctx *ctx, uint32_t log2_records) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  if (log2_records > 1 && (log2_records < kad::TABLE_MIN_BITS || log2_records > kad::TABLE_MAX_BITS))
    return fail(KAD_EINVAL, "slot tables hold 2^%u to 2^%u records", kad::TABLE_MIN_BITS,
                kad::TABLE_MAX_BITS);
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipDeviceSynchronize());  // no launch may still use the slots
  ctx->table_knob = log2_records;
  ctx->slots = 0;  // laid out again (and the wide-count arena after them) on next use
  ctx->slot_n = 0;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_get_table(kad_ctx *ctx, uint32_t *log2_records, uint32_t *slots,
                             uint32_t *wide_slots) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  if (log2_records) *log2_records = ctx->slots ? ctx->slot_hbits : 0;
  if (slots) *slots = ctx->slots;
  if (wide_slots) *wide_slots = ctx->slots ? kad::wide_slot_count(ctx) : 0;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_set_exec(kad_ctx *ctx, uint32_t mode) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  if (mode > KAD_EXEC_PLAIN) return fail(KAD_EINVAL, "unknown launch mode %u", mode);
  kad::CtxClaim claim(ctx);
  if (!claim.ok()) return fail(KAD_EBUSY, "the context is in use (another call or a server)");
  ctx->exec = mode;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_get_exec(kad_ctx *ctx, uint32_t *mode, uint64_t *records, uint64_t *replays) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  if (mode) *mode = ctx->exec;
  if (records) *records = ctx->chain_records.load();
  if (replays) *replays = ctx->chain_replays.load();
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

kad_status kad_ctx_get_timing(kad_ctx *ctx, uint64_t *launches, uint64_t *samples,
                              double *seconds, uint64_t *arcs, uint64_t *nodes, uint64_t *hits) try {
  if (!ctx) return fail(KAD_EINVAL, "NULL context");
  if (launches) *launches = ctx->t_launches;
  if (samples) *samples = ctx->t_samples;
  if (seconds) *seconds = ctx->t_seconds;
  if (arcs) *arcs = ctx->t_arcs;
  if (nodes) *nodes = ctx->t_nodes;
  if (hits) *hits = ctx->t_hits;
  return KAD_OK;
} catch (...) {
  return kad::status_of_exception();
}

}  // extern "C"
