// HIP kernels of the sampled-betweenness hot path, written for CDNA4 (gfx950).
//
// sampler_kernel: one workgroup per sample (Borassi & Natale, section 4 "Balanced
//   Bidirectional BFS"; pair and path distribution of section 2).  A persistent
//   grid pulls sample ids from a counter; everything random is a Philox4x64-10
//   draw keyed by (seed, phase, sample id, purpose, step), so results do not
//   depend on which workgroup runs which sample.
//
//   Each level expansion is split in two scans of the frontier's rows:
//     touch scan     -- for every arc, test its head against the other side's
//                       frontier (an LDS bit filter, confirmed by the node's tag)
//                       and collect the candidate edges;
//     discovery scan -- only when the two searches did not touch: claim unseen
//                       heads for the next level (compare-and-swap on the tag),
//                       add the 128-bit path counts, append the new frontier with
//                       wave ballots.
//   The expansion that meets -- normally the largest one -- therefore costs
//   coalesced row reads and LDS probes only.
//
// Hit reductions (interior nodes of the sampled paths -> per-node counters), three kinds:
//   hit_partition/hit_tile -- per node-id tile, an LDS histogram whose cells are added to
//     the counters by the one thread that claims each cell: no atomics on the counters
//     (large calls and subtractions);
//   hit_atomic_kernel -- one device atomic add per hit (calls of at most 2^17 hits);
//   iv_count/iv_prefix/iv_snap -- every check interval of a batch at once: per-interval
//     hit counts by device atomics on scratch, then one owner per node adds them to its
//     counter interval by interval.
//   The atomic forms were measured faster on the run's critical path.
#include <algorithm>
#include <mutex>

#include "kad_device.h"

namespace kad {
namespace {

// The sampler is compiled for workgroups of 64, 128 and 256 threads (one sample per
// workgroup); the launcher picks one per launch.
constexpr int WAVE = 64;
constexpr int FILTER_LOG2 = 15;
constexpr int FILTER_WORDS = (1 << FILTER_LOG2) / 32;
constexpr int PI_LDS = 256;  // candidate edges kept in LDS; more spill to the slot buffer
constexpr uint32_t MAX_ATTEMPTS = 64;
constexpr int MAXLEV = 32;     // levels per side whose node lists are remembered
constexpr int MATCH_CAP = 48;  // predecessor candidates a backtracking wave keeps in LDS
constexpr uint32_t MAX_HIT_TILES = MAX_HIT_TILES_PUBLIC;


// ------------------------------------------------------------------ Philox4x64-10
// Salmon et al., SC'11: ten rounds of two 64x64->128 multiplications; the key is
// bumped by two Weyl constants between rounds.
constexpr uint64_t PH_M0 = 0xD2E7470EE14C6C93ULL;
constexpr uint64_t PH_M1 = 0xCA5A826395121157ULL;
constexpr uint64_t PH_W0 = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t PH_W1 = 0xBB67AE8584CAA73BULL;

__device__ __forceinline__ void philox4(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PH_W0;
      k1 += PH_W1;
    }
    const uint64_t lo0 = PH_M0 * c0, hi0 = __umul64hi(PH_M0, c0);
    const uint64_t lo1 = PH_M1 * c2, hi1 = __umul64hi(PH_M1, c2);
    const uint64_t y0 = hi1 ^ c1 ^ k0;
    const uint64_t y2 = hi0 ^ c3 ^ k1;
    c0 = y0;
    c1 = lo1;
    c2 = y2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// The first two output words (all that draws of up to 128 bits use).
__device__ __forceinline__ void philox2(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1, uint64_t &o0, uint64_t &o1) {
  uint64_t w[4];
  philox4(c0, c1, c2, c3, k0, k1, w);
  o0 = w[0];
  o1 = w[1];
}

__device__ __forceinline__ uint64_t stream_word(uint32_t phase, uint32_t purpose, uint64_t step) {
  return ((uint64_t)phase << 56) | ((uint64_t)purpose << 48) | (step & 0xFFFFFFFFFFFFULL);
}

enum : uint32_t { P_S = 0, P_T = 1, P_EDGE = 2, P_BACK_S = 3, P_BACK_T = 4 };

// ------------------------------------------------------------------ 128-bit naturals
struct u128 {
  uint64_t lo, hi;
};

__device__ __forceinline__ bool lt128(u128 a, u128 b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

__device__ __forceinline__ u128 add128(u128 a, u128 b, bool &ovf) {
  u128 r;
  r.lo = a.lo + b.lo;
  const uint64_t c = r.lo < a.lo ? 1u : 0u;
  const uint64_t t = a.hi + b.hi;
  ovf |= t < a.hi;
  r.hi = t + c;
  ovf |= r.hi < t;
  return r;
}

__device__ __forceinline__ u128 sub128(u128 a, u128 b) {  // a >= b
  u128 r;
  r.lo = a.lo - b.lo;
  r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
  return r;
}

__device__ __forceinline__ u128 mul128(u128 a, u128 b, bool &ovf) {
  if (a.hi != 0 && b.hi != 0) {
    ovf = true;
    return u128{0, 0};
  }
  u128 r;
  r.lo = a.lo * b.lo;
  const uint64_t h = __umul64hi(a.lo, b.lo);
  const uint64_t x1 = a.lo * b.hi, x1h = __umul64hi(a.lo, b.hi);
  const uint64_t x2 = a.hi * b.lo, x2h = __umul64hi(a.hi, b.lo);
  ovf |= (x1h | x2h) != 0;
  uint64_t cross = x1 + x2;
  ovf |= cross < x1;
  r.hi = h + cross;
  ovf |= r.hi < h;
  return r;
}

__device__ __forceinline__ uint32_t bitlen128(u128 x) {
  if (x.hi) return 128u - (uint32_t)__clzll(x.hi);
  if (x.lo) return 64u - (uint32_t)__clzll(x.lo);
  return 0u;
}

// An integer uniform in [0, bound), bound >= 1: W = bitlength(bound - 1); attempt a
// takes ceil(W/64) words of block 0 of counter (i, sword, a, 0), least-significant
// first, keeps W bits and accepts the value if it is below the bound.
__device__ u128 uniform_below(u128 bound, uint64_t seed, uint64_t i, uint64_t sword,
                              uint32_t &flags) {
  if (bound.hi == 0 && bound.lo == 1) return u128{0, 0};
  const u128 bm1 = sub128(bound, u128{1, 0});
  const uint32_t W = bitlen128(bm1);
  const uint32_t q = (W + 63) / 64;
  const uint32_t top = W - 64 * (q - 1);
  const uint64_t mask = top == 64 ? ~0ULL : ((1ULL << top) - 1);
  for (uint32_t a = 0; a < MAX_ATTEMPTS; ++a) {
    uint64_t o0, o1;
    philox2(i, sword, a, 0, seed, 0, o0, o1);
    u128 x;
    if (q == 1) {
      x.lo = o0 & mask;
      x.hi = 0;
    } else {
      x.lo = o0;
      x.hi = o1 & mask;
    }
    if (lt128(x, bound)) return x;
  }
  flags |= FLAG_RNG;
  return u128{0, 0};
}

// ------------------------------------------------------------------ memory helpers
// A slot's node records are touched only by the workgroup that owns the slot,
// so every atomic and every load that must observe one is workgroup-scoped: it stays
// in the CU's XCD (no cross-XCD coherence traffic), and __syncthreads orders it.
// Between launches the slot state is all-zero, whichever XCD ran it last.
//
// A node's state in a slot is one record of REC_WORDS words (32 bytes, so four nodes
// share a 128-byte line and a node's tag and count share one): word 0 the tag, word 1
// the wide-count kernel's node position, words 2-5 the 128-bit path count (low, high).
__device__ __forceinline__ uint32_t *tag_of(uint32_t *rec, uint32_t v) {
  return rec + (size_t)REC_WORDS * v;
}
__device__ __forceinline__ const uint32_t *tag_of(const uint32_t *rec, uint32_t v) {
  return rec + (size_t)REC_WORDS * v;
}
__device__ __forceinline__ uint32_t *pos_of(uint32_t *rec, uint32_t v) {
  return rec + (size_t)REC_WORDS * v + 1;
}
__device__ __forceinline__ uint64_t *sig_of(uint32_t *rec, uint32_t v) {
  return reinterpret_cast<uint64_t *>(rec + (size_t)REC_WORDS * v + 2);
}
__device__ __forceinline__ const uint64_t *sig_of(const uint32_t *rec, uint32_t v) {
  return reinterpret_cast<const uint64_t *>(rec + (size_t)REC_WORDS * v + 2);
}
__device__ __forceinline__ uint32_t ld_tag(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ u128 ld_sig(const uint32_t *rec, uint32_t v) {
  const uint64_t *p = sig_of(rec, v);
  u128 r;
  r.lo = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  r.hi = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return r;
}
__device__ __forceinline__ uint32_t cas_tag(uint32_t *p, uint32_t expect, uint32_t want) {
  __hip_atomic_compare_exchange_strong(p, &expect, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
  return expect;  // the value found (== the old expectation on success)
}
__device__ __forceinline__ uint64_t add_u64(uint64_t *p, uint64_t x) {
  return __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------------------ slot tables
// A sampler slot keeps its records in one of two layouts (SlotState::hbits):
//   dense  -- node v's record at index v, one record per node of the graph;
//   hashed -- a table of 2^hbits records.  Node v sits at the first index of
//             home(v), home(v) + 1, ... (mod the table size) whose word 1 holds v + 1,
//             at most MAX_PROBE steps from home(v).  One 64-bit compare-and-swap on
//             words 0-1 (tag, key) places a node and claims it at once.  A node that
//             cannot be placed within MAX_PROBE steps gives its sample FLAG_CAPACITY:
//             the wide-count kernel, whose records are dense, samples it again.  So a
//             lookup that meets neither its key nor an empty record within MAX_PROBE
//             steps knows the node has no record.
// Entries are never removed while a sample runs; its reset clears every record it placed
// (the reached list keeps each node's index beside its id).
constexpr uint32_t MAX_PROBE = 32;
constexpr uint32_t NO_REC = 0xFFFFFFFFu;

struct Recs {
  uint32_t *rec;
  uint32_t hbits;  // hashed layouts only: log2 of the table size
  __device__ __forceinline__ uint32_t home(uint32_t v) const {
    return (v * 2654435761u) >> (32 - hbits);
  }
  __device__ __forceinline__ uint32_t mask() const { return (1u << hbits) - 1u; }
  __device__ __forceinline__ uint64_t *word(uint32_t idx) const {
    return reinterpret_cast<uint64_t *>(rec + (size_t)REC_WORDS * idx);
  }
};
__device__ __forceinline__ uint64_t rec_word(uint32_t v, uint32_t tag) {
  return ((uint64_t)(v + 1u) << 32) | tag;
}
__device__ __forceinline__ uint64_t ld_word(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t cas_word(uint64_t *p, uint64_t expect, uint64_t want) {
  __hip_atomic_compare_exchange_strong(p, &expect, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
  return expect;  // the word found (0 on success)
}
// v's word and index (0 and NO_REC: no record).
__device__ __forceinline__ uint64_t rec_find(const Recs &R, uint32_t v, uint32_t &h) {
  const uint32_t key = v + 1u, m = R.mask();
  h = R.home(v);
  for (uint32_t p = 0; p < MAX_PROBE; ++p, h = (h + 1u) & m) {
    const uint64_t x = ld_word(R.word(h));
    const uint32_t k = (uint32_t)(x >> 32);
    if (k == key) return x;
    if (k == 0) break;
  }
  h = NO_REC;
  return 0;
}
// Record index of node v in a table (NO_REC: none).  Out of line: its probe loop, inlined
// into the 128-bit arithmetic of the callers, would take their registers.
__device__ __noinline__ uint32_t rec_index(uint32_t *rec, uint32_t hbits, uint32_t v) {
  uint32_t h;
  (void)rec_find(Recs{rec, hbits}, v, h);
  return h;
}
// The 128-bit count of node v, which has a record (zero, and FLAG_CAPACITY in fl, if not).
template <bool HASHED>
__device__ __forceinline__ u128 node_sig(const Recs &R, uint32_t v, uint32_t &fl) {
  if (!HASHED) return ld_sig(R.rec, v);
  const uint32_t h = rec_index(R.rec, R.hbits, v);
  if (h == NO_REC) {
    fl |= FLAG_CAPACITY;
    return u128{0, 0};
  }
  return ld_sig(R.rec, h);
}

__device__ __forceinline__ uint32_t filter_bit(uint32_t w) {
  return (w * 2654435761u) >> (32 - FILTER_LOG2);
}

// Exact set of node ids in SLOTS words of LDS (open addressing, linear probing), kept
// at most half full so that every probe sequence reaches an empty word.
constexpr uint32_t FSET_EMPTY = 0xFFFFFFFFu;  // never a node id
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
template <int SLOTS>
__device__ __forceinline__ uint32_t fset_slot(uint32_t w) {
  return (w * 0x85EBCA6Bu) >> (32 - ilog2(SLOTS));
}
template <int SLOTS>
__device__ __forceinline__ void fset_insert(uint32_t *fs, uint32_t w) {
  uint32_t h = fset_slot<SLOTS>(w);
  while (atomicCAS(&fs[h], FSET_EMPTY, w) != FSET_EMPTY) h = (h + 1) & (SLOTS - 1);
}
template <int SLOTS>
__device__ __forceinline__ bool fset_has(const uint32_t *fs, uint32_t w) {
  uint32_t h = fset_slot<SLOTS>(w);
  for (;;) {
    const uint32_t x = fs[h];
    if (x == w) return true;
    if (x == FSET_EMPTY) return false;
    h = (h + 1) & (SLOTS - 1);
  }
}

// ------------------------------------------------------------------ wave / block scans
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ uint32_t wave_incl_u32(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, WAVE);
    if (lane >= (uint32_t)d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

__device__ __forceinline__ u128 wave_incl_u128(u128 v, bool &ovf) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint64_t olo = __shfl_up(v.lo, d, WAVE);
    const uint64_t ohi = __shfl_up(v.hi, d, WAVE);
    if (lane >= (uint32_t)d) v = add128(v, u128{olo, ohi}, ovf);
  }
  return v;
}

template <int BLOCK>
struct Lds {
  static constexpr int NWAVES = BLOCK / WAVE;
  static constexpr int CHUNK = 2 * BLOCK;  // frontier nodes staged per pass (2 per thread)
  // The frontier bit filter; once the searches have met, its words (and those of the
  // count staging area below) hold the candidate edges while they are sorted.
  union {
    uint32_t filter[FILTER_WORDS];
    uint64_t sort_lo[FILTER_WORDS / 2];
  };
  uint64_t pi[PI_LDS];
  // The path counts of a chunk's rows (discovery scans); during a touch scan the same
  // bytes hold the other side's frontier as an exact hash set.
  union {
    struct {
      uint64_t c_sig_lo[CHUNK];
      uint64_t c_sig_hi[CHUNK];
    };
    uint32_t fset[4 * CHUNK];
    uint64_t sort_hi[2 * CHUNK];
  };
  uint32_t c_node[CHUNK];
  uint32_t c_off[CHUNK];  // short rows: row start minus the row's first position in the
                          // chunk's arc space; long rows: the row start
  uint32_t c_deg[CHUNK];
  static constexpr int MASK_WORDS = BLOCK / 4;  // the widest window: 8 arcs per thread
  uint32_t wmask[3][MASK_WORDS];  // row starts of an arc window, one bit per arc (triple-buffered)
  uint32_t wfirst[3];       // the row that holds a window's first arc
  uint32_t red32[NWAVES + 1];
  uint32_t red32b[NWAVES + 1];
  uint64_t red_lo[NWAVES];
  uint64_t red_hi[NWAVES];
  uint64_t deg[2];
  uint32_t st0[2];  // row starts of s (out-row) and t (in-row)
  uint64_t arcs;
  uint64_t new_deg;
  uint64_t r_lo, r_hi, wkey;
  uint32_t rfl;
  uint32_t k, s, t, seg;
  uint32_t fb[2], fe[2], lvl[2];
  uint32_t nvis, pi_count, flags, win;
  uint32_t ovf_any;
  uint32_t needed;  // nodes on completed levels (the reached set the method needs)
  uint32_t seg_lo[2][MAXLEV], seg_hi[2][MAXLEV];  // level l of a side = visit[seg_lo, seg_hi)
};

// Backtracking scratch of one wave, carved out of the candidate-edge staging area
// (free once the meeting edge is chosen).
struct MatchScratch {
  uint32_t id[MATCH_CAP];
  uint64_t lo[MATCH_CAP];
  uint64_t hi[MATCH_CAP];
};
static_assert(2 * sizeof(MatchScratch) <= PI_LDS * sizeof(uint64_t), "scratch fits the staging area");

// Exclusive block scan of one value per thread; *total gets the block sum.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_u32(Lds<BLOCK> &L, uint32_t v, uint32_t &total) {
  constexpr int NWAVES = BLOCK / WAVE;
  const uint32_t lane = lane_id(), wid = threadIdx.x / WAVE;
  const uint32_t inc = wave_incl_u32(v);
  if (lane == WAVE - 1) L.red32[wid] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int q = 0; q < NWAVES; ++q) {
    const uint32_t x = L.red32[q];
    if ((uint32_t)q < wid) before += x;
    all += x;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

// Exclusive block scan of two values per thread at once.
template <int BLOCK>
__device__ __forceinline__ void block_excl2_u32(Lds<BLOCK> &L, uint32_t a, uint32_t b,
                                                uint32_t &ea, uint32_t &eb, uint32_t &ta,
                                                uint32_t &tb) {
  constexpr int NWAVES = BLOCK / WAVE;
  const uint32_t lane = lane_id(), wid = threadIdx.x / WAVE;
  const uint32_t ia = wave_incl_u32(a), ib = wave_incl_u32(b);
  if (lane == WAVE - 1) {
    L.red32[wid] = ia;
    L.red32b[wid] = ib;
  }
  __syncthreads();
  uint32_t ba = 0, bb = 0, aa = 0, ab = 0;
#pragma unroll
  for (int q = 0; q < NWAVES; ++q) {
    const uint32_t xa = L.red32[q], xb = L.red32b[q];
    if ((uint32_t)q < wid) {
      ba += xa;
      bb += xb;
    }
    aa += xa;
    ab += xb;
  }
  __syncthreads();
  ta = aa;
  tb = ab;
  ea = ba + ia - a;
  eb = bb + ib - b;
}

// Inclusive block scan of 128-bit values; *total gets the block sum.
template <int BLOCK>
__device__ __forceinline__ u128 block_incl_u128(Lds<BLOCK> &L, u128 v, u128 &total, bool &ovf) {
  constexpr int NWAVES = BLOCK / WAVE;
  const uint32_t lane = lane_id(), wid = threadIdx.x / WAVE;
  u128 inc = wave_incl_u128(v, ovf);
  if (lane == WAVE - 1) {
    L.red_lo[wid] = inc.lo;
    L.red_hi[wid] = inc.hi;
  }
  __syncthreads();
  u128 before{0, 0}, all{0, 0};
#pragma unroll
  for (int q = 0; q < NWAVES; ++q) {
    const u128 x{L.red_lo[q], L.red_hi[q]};
    if ((uint32_t)q < wid) before = add128(before, x, ovf);
    all = add128(all, x, ovf);
  }
  __syncthreads();
  total = all;
  return add128(before, inc, ovf);
}

// Wave-aggregated append of the lanes with `pred` to an LDS-counted list.
__device__ __forceinline__ uint32_t wave_reserve(bool pred, uint32_t *counter, uint32_t &rank) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return 0xFFFFFFFFu;
  const uint32_t lane = lane_id();
  const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, leader, WAVE);
  rank = (uint32_t)__popcll(mask & ((1ULL << lane) - 1ULL));
  return base;
}

// Whether a touch scan tests a long row of d arcs against the other side's frontier
// (om nodes) by binary searches instead of reading it: when the searches read fewer
// lines.  The row is sorted, so each search finds one frontier node or proves it
// absent; om searches read about om * (log2(d) - 4) lines below the levels they share
// (4-byte ids, 128-byte lines), reading the row takes d / 32 lines.  (All searches of
// a chunk form one chain of about log2(d) dependent loads; the row takes
// d / (BLOCK * U) rounds.)  The edges found are the same; their order in the candidate
// list is not, and the choice among them depends only on their keys.
__device__ __forceinline__ bool touch_by_search(uint32_t d, uint32_t om) {
  if (d < 1024u || om == 0) return false;
  const uint32_t depth = 27u - (uint32_t)__clz(d);  // floor(log2 d) - 4, at least 6
  return (uint64_t)om * depth * 32u < (uint64_t)d;
}

// Touch: meeting test only (filter + tag).  Discover: next-level claims and counts only.
// Both: the meeting test by tag and the discovery in one pass (small expansions).
enum class Scan { Touch, Discover, Both };

// One pass over the rows of frontier [fb, fe), chunked through LDS.
//
// Rows of at least one window of arcs ("long" rows) are walked by the waves piece by
// piece: a piece is WAVE * U consecutive arcs of one row, so every arc's row is known
// and a long row costs no bookkeeping.  The other rows of nonzero degree ("short"
// rows; rows of degree zero own no arcs and are dropped) are laid end to end in one
// arc space [0, tot) and walked in windows of BLOCK * U: lane l of wave w takes arcs
// e0 + w*WAVE*U + q*WAVE + l, q < U.  The short row that owns an arc is found without
// a search: every short row that starts inside the window sets the bit of its first
// position in an LDS mask, and the owner of position p is the window's first row plus
// the number of starts in (0, p] -- a popcount over the mask.  The masks are
// triple-buffered so that a window takes one barrier: window k sets its bits in mask
// k mod 3 and clears mask (k+1) mod 3, which every wave finished reading before the
// barrier of window k-1.  wk is the window counter (mod 3), carried from call to call.
// Short rows take the chunk slots from the front, long rows from the back, and below
// them (touch scans only) the long rows that are searched for the other frontier's om
// nodes visit[ob, ob + om) rather than read (touch_by_search).
// HASHED: the slot's records form a table of 2^hbits (see Recs); vh[j] is the record
// index of visit[j].
template <int BLOCK, Scan MODE, bool HASHED>
__device__ __forceinline__ void scan_frontier(Lds<BLOCK> &L, const GraphDev &g, uint32_t me,
                                              uint32_t fb, uint32_t fe, uint32_t *rec,
                                              uint32_t hbits, uint32_t *visit, uint32_t *vh,
                                              uint64_t *gpi, uint32_t pi_cap,
                                              uint32_t other_tag, uint32_t next_tag,
                                              bool &ovf, uint32_t &wk, bool exact, bool first,
                                              uint32_t ob = 0, uint32_t om = 0) {
  const Recs R{rec, hbits};
  constexpr int CHUNK = 2 * BLOCK;
  // arcs per lane per window or piece: a window costs a few dependent round trips
  // whatever its size; wider touch windows than 8 run out of registers
  // (hashed records: four, the probes' indices and words take the registers)
  constexpr int U = MODE == Scan::Touch ? (HASHED ? 4 : 8) : (MODE == Scan::Discover ? 4 : 2);
  constexpr uint32_t WIN = BLOCK * U;
  constexpr uint32_t PIECE = WAVE * U;
  constexpr uint32_t NWAVES = BLOCK / WAVE;
  constexpr uint32_t NWORDS = WIN / 32;
  static_assert(NWORDS <= (uint32_t)Lds<BLOCK>::MASK_WORDS && NWORDS <= (uint32_t)WAVE &&
                    WIN % 64 == 0,
                "a window's mask fits its buffer and one wave");
  const uint32_t tid = threadIdx.x, lane = lane_id();
  const uint32_t wid = __builtin_amdgcn_readfirstlane(tid / WAVE);
  const uint32_t *rp = me == 0 ? g.row : g.rrow;
  const uint32_t *cl = me == 0 ? g.col : g.rcol;
  // bits of the mask word at or below this lane's position (positions of a wave's
  // group are 64-aligned, so a lane always sits at bit lane mod 32)
  const uint32_t below = ((1u << (lane & 31)) << 1) - 1u;

  // The arcs ww[q] of this lane (bit q of vm: the arc exists), owned by the chunk rows
  // owner(q): the touch test or the discovery step.  Every stage first issues the loads
  // or atomics of all U arcs and only then uses their results, so a lane keeps U memory
  // requests in flight instead of waiting on one arc at a time.
  auto process = [&](const uint32_t (&ww)[U], uint32_t vm, auto owner) {
    if (MODE == Scan::Touch) {
      // filter probes; an arc that passes is confirmed in the exact set when the other
      // frontier has one, else by its tag (the tag loads of all arcs go out together)
      uint32_t fword[U];
#pragma unroll
      for (int q = 0; q < U; ++q) fword[q] = L.filter[filter_bit(ww[q]) >> 5];
      uint32_t pass = 0, hitm = 0;
#pragma unroll
      for (int q = 0; q < U; ++q)
        pass |= (fword[q] >> (filter_bit(ww[q]) & 31)) & (vm >> q) & 1u ? 1u << q : 0u;
      if (exact) {
#pragma unroll
        for (int q = 0; q < U; ++q)
          if ((pass >> q) & 1u) hitm |= fset_has<4 * CHUNK>(L.fset, ww[q]) ? 1u << q : 0u;
      } else if (HASHED) {
        // every round of probes goes out together: first the home records, then the next
        // record of each arc whose probe met another node (rare at the tables' fill)
        uint64_t x[U];
        uint32_t h[U], open = pass;  // open bit q: arc q not yet resolved
#pragma unroll
        for (int q = 0; q < U; ++q) {
          h[q] = R.home(ww[q]);
          x[q] = (open >> q) & 1u ? ld_word(R.word(h[q])) : 0ull;
        }
        for (uint32_t p = 0;; ++p) {
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const uint32_t k = (uint32_t)(x[q] >> 32);
            if (k == 0 || k == ww[q] + 1u) open &= ~(1u << q);
          }
          if (open == 0 || p + 1 == MAX_PROBE) break;
#pragma unroll
          for (int q = 0; q < U; ++q) {
            if ((open >> q) & 1u) {
              h[q] = (h[q] + 1u) & R.mask();
              x[q] = ld_word(R.word(h[q]));
            }
          }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
          hitm |= (uint32_t)(x[q] >> 32) == ww[q] + 1u && (uint32_t)x[q] == other_tag ? 1u << q : 0u;
      } else {
        uint32_t tg[U];
#pragma unroll
        for (int q = 0; q < U; ++q) tg[q] = (pass >> q) & 1u ? ld_tag(tag_of(rec, ww[q])) : 0u;
#pragma unroll
        for (int q = 0; q < U; ++q) hitm |= tg[q] == other_tag ? 1u << q : 0u;  // never 0
      }
      if (__ballot(hitm != 0)) {  // uniform: some lane of this wave found candidates
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const bool hit = (hitm >> q) & 1u;
          uint32_t rank = 0;
          const uint32_t base = wave_reserve(hit, &L.pi_count, rank);
          if (hit) {
            const uint32_t u = L.c_node[owner(q)], w = ww[q];
            const uint64_t key = me == 0 ? (((uint64_t)u << 32) | w) : (((uint64_t)w << 32) | u);
            const uint32_t idx = base + rank;
            if (idx < (uint32_t)PI_LDS) L.pi[idx] = key;
            else if (idx < pi_cap) gpi[idx] = key;
          }
        }
      }
    } else {
      // Claims: one compare-and-swap per arc returns the head's tag as it was (0 if
      // unseen, then this arc claimed it; next_tag if another arc of this level did;
      // other_tag if the head is in the other side's frontier).
      // HASHED: the claim places the head in the table (at[q]: its record index); the
      // home probes of all arcs go out together, a probe that meets another node
      // continues alone, and a head that finds no room within MAX_PROBE steps leaves the
      // sample to the wide-count kernel
      uint32_t tg[U], at[U], dm = 0;  // dm bit q: this lane's arc of group q claimed its head
      if (HASHED) {
        // every round of compare-and-swaps goes out together: first at the home records,
        // then at the next record of each head whose attempt met another node
        uint64_t x[U];
        uint32_t open = vm;  // open bit q: head q neither placed nor found yet
#pragma unroll
        for (int q = 0; q < U; ++q) {
          at[q] = R.home(ww[q]);
          x[q] = (open >> q) & 1u ? cas_word(R.word(at[q]), 0, rec_word(ww[q], next_tag)) : 0ull;
        }
        for (uint32_t p = 0;; ++p) {
#pragma unroll
          for (int q = 0; q < U; ++q)
            if (x[q] == 0 || (uint32_t)(x[q] >> 32) == ww[q] + 1u) open &= ~(1u << q);
          if (open == 0 || p + 1 == MAX_PROBE) break;
#pragma unroll
          for (int q = 0; q < U; ++q) {
            if ((open >> q) & 1u) {
              at[q] = (at[q] + 1u) & R.mask();
              x[q] = cas_word(R.word(at[q]), 0, rec_word(ww[q], next_tag));
            }
          }
        }
        if (open) atomicOr(&L.flags, FLAG_CAPACITY);  // no room within MAX_PROBE records
#pragma unroll
        for (int q = 0; q < U; ++q) {
          tg[q] = 0;
          if (((vm & ~open) >> q) & 1u) {
            dm |= x[q] == 0 ? 1u << q : 0u;
            tg[q] = x[q] == 0 ? next_tag : (uint32_t)x[q];
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < U; ++q) {
          tg[q] = 0;
          if ((vm >> q) & 1u) {
            const uint32_t old = cas_tag(tag_of(rec, ww[q]), 0u, next_tag);
            dm |= old == 0 ? 1u << q : 0u;
            tg[q] = old == 0 ? next_tag : old;
          }
        }
      }
      // sigma(w) += sigma(u) on the low words, the appends of the claimed heads and
      // the loads of their degrees all go out before any result is used; the carries
      // into the high words follow
      uint64_t old_lo[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        old_lo[q] = 0;
        if (tg[q] == next_tag)
          old_lo[q] = add_u64(sig_of(rec, HASHED ? at[q] : ww[q]), L.c_sig_lo[owner(q)]);
      }
      if (MODE == Scan::Both) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const bool hit = tg[q] == other_tag;  // never 0
          uint32_t prank = 0;
          const uint32_t pbase = wave_reserve(hit, &L.pi_count, prank);
          if (hit) {
            const uint32_t u = L.c_node[owner(q)], w = ww[q];
            const uint64_t key = me == 0 ? (((uint64_t)u << 32) | w) : (((uint64_t)w << 32) | u);
            const uint32_t idx = pbase + prank;
            if (idx < (uint32_t)PI_LDS) L.pi[idx] = key;
            else if (idx < pi_cap) gpi[idx] = key;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const bool disc = (dm >> q) & 1u;
        uint32_t rank = 0;
        const uint32_t base = wave_reserve(disc, &L.nvis, rank);
        if (disc) {
          visit[base + rank] = ww[q];
          if (HASHED) vh[base + rank] = at[q];
        }
      }
      if (__ballot(dm != 0)) {  // uniform: some lane of this wave discovered a node
        uint64_t dg = 0;
#pragma unroll
        for (int q = 0; q < U; ++q)
          if ((dm >> q) & 1u) dg += (uint64_t)(rp[ww[q] + 1] - rp[ww[q]]);
        const uint64_t sum = wave_sum_u64(dg);
        if (lane == 0) atomicAdd((unsigned long long *)&L.new_deg, (unsigned long long)sum);
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (tg[q] == next_tag) {
          const uint32_t j = owner(q);
          const uint64_t xlo = L.c_sig_lo[j], xhi = L.c_sig_hi[j];
          const uint64_t add = xhi + ((old_lo[q] + xlo < old_lo[q]) ? 1u : 0u);
          ovf |= add < xhi;
          if (add != 0) {
            const uint64_t oh = add_u64(sig_of(rec, HASHED ? at[q] : ww[q]) + 1, add);
            ovf |= oh + add < oh;
          }
        }
      }
    }
  };

  for (uint32_t cb = fb; cb < fe; cb += CHUNK) {
    const uint32_t m = min((uint32_t)CHUNK, fe - cb);
    uint32_t u[2] = {0, 0}, st[2] = {0, 0}, d[2] = {0, 0};
    u128 su[2] = {{0, 0}, {0, 0}};
    if (first) {
      // the endpoint alone (level 0): its row and count are known, nothing to load
      if (tid == 0) {
        u[0] = me == 0 ? L.s : L.t;
        st[0] = L.st0[me];
        d[0] = (uint32_t)L.deg[me];
        su[0] = u128{1, 0};
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint32_t j = 2 * tid + q;
        if (j < m) {
          u[q] = visit[cb + j];
          st[q] = rp[u[q]];
          d[q] = rp[u[q] + 1] - st[q];
          if (MODE != Scan::Touch) su[q] = ld_sig(rec, HASHED ? vh[cb + j] : u[q]);
        }
      }
    }
    // classes: 0 none, 1 short, 2 long, 3 searched (an endpoint's row, alone, is never
    // short: it needs no window bookkeeping)
    uint32_t cls[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      cls[q] = d[q] == 0 ? 0u : (d[q] < WIN && !first ? 1u : 2u);
      if (MODE == Scan::Touch && cls[q] == 2 && touch_by_search(d[q], om)) cls[q] = 3;
    }
    // per-class row counts in three 10-bit fields (a chunk has at most 512 rows)
    static_assert(CHUNK < 1024, "row counts fit their fields");
    constexpr uint32_t F_LONG = 1u << 10, F_SEARCH = 1u << 20;
    const uint32_t sarcs = (cls[0] == 1 ? d[0] : 0u) + (cls[1] == 1 ? d[1] : 0u);
    uint32_t cnts = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q)
      cnts += cls[q] == 1 ? 1u : (cls[q] == 2 ? F_LONG : (cls[q] == 3 ? F_SEARCH : 0u));
    uint32_t ex = 0, cx = 0, tot, ncx;
    if (first) {  // one row, held by thread 0: the scan's results are known
      const uint32_t d0 = (uint32_t)L.deg[me];
      tot = 0;
      ncx = d0 == 0 ? 0u
                    : (MODE == Scan::Touch && touch_by_search(d0, om) ? F_SEARCH : F_LONG);
    } else {
      block_excl2_u32(L, sarcs, cnts, ex, cx, tot, ncx);
    }
    const uint32_t nlong = (ncx >> 10) & 1023u, nsearch = ncx >> 20;
    // this thread's rows: chunk slot and (short rows) first position in the arc space
    uint32_t slot[2], pos[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t same = q == 1 && cls[0] == cls[1] ? 1u : 0u;  // row 0 goes first
      slot[q] = cls[q] == 1   ? (cx & 1023u) + same
                : cls[q] == 2 ? CHUNK - 1 - ((cx >> 10) & 1023u) - same
                              : CHUNK - 1 - nlong - (cx >> 20) - same;
    }
    pos[0] = ex;
    pos[1] = ex + (cls[0] == 1 ? d[0] : 0u);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (cls[q] != 0) {
        L.c_node[slot[q]] = u[q];
        L.c_off[slot[q]] = cls[q] == 1 ? st[q] - pos[q] : st[q];
        L.c_deg[slot[q]] = d[q];
        if (MODE != Scan::Touch) {
          L.c_sig_lo[slot[q]] = su[q].lo;
          L.c_sig_hi[slot[q]] = su[q].hi;
        }
      }
    }

    if (nlong + nsearch > 0) __syncthreads();
    // ---- searched rows: one lane per (row, other-frontier node) pair
    if (MODE == Scan::Touch && nsearch > 0) {
      const uint32_t pairs = nsearch * om;
      for (uint32_t p0 = 0; p0 < pairs; p0 += BLOCK) {
        const uint32_t p = p0 + tid;
        bool hit = false;
        uint32_t u = 0, w = 0;
        if (p < pairs) {
          const uint32_t r = p / om;
          const uint32_t sl = CHUNK - 1 - nlong - r;
          const uint32_t rst = L.c_off[sl], rd = L.c_deg[sl];
          w = visit[ob + (p - r * om)];
          u = L.c_node[sl];
          uint32_t lo = 0, len = rd;  // first position whose id is not below w
          while (len > 0) {
            const uint32_t half = len >> 1;
            if (cl[rst + lo + half] < w) {
              lo += half + 1;
              len -= half + 1;
            } else {
              len = half;
            }
          }
          hit = lo < rd && cl[rst + lo] == w;
        }
        uint32_t rank = 0;
        const uint32_t base = wave_reserve(hit, &L.pi_count, rank);
        if (hit) {
          const uint64_t key = me == 0 ? (((uint64_t)u << 32) | w) : (((uint64_t)w << 32) | u);
          const uint32_t idx = base + rank;
          if (idx < (uint32_t)PI_LDS) L.pi[idx] = key;
          else if (idx < pi_cap) gpi[idx] = key;
        }
      }
    }

    // ---- long rows, piece by piece (no barrier between pieces); the row loads of a
    // wave's next piece go out before its current piece is tested
    if (nlong > 0) {
      for (uint32_t r = 0; r < nlong; ++r) {
        const uint32_t sl = CHUNK - 1 - r;
        const uint32_t rst = L.c_off[sl], rd = L.c_deg[sl];
        uint32_t nx[U];
        uint32_t off = wid * PIECE;
        if (off < rd) {
#pragma unroll
          for (int q = 0; q < U; ++q) nx[q] = cl[rst + min(off + q * WAVE + lane, rd - 1)];
        }
        for (; off < rd; off += NWAVES * PIECE) {
          uint32_t ww[U], vm = 0;
#pragma unroll
          for (int q = 0; q < U; ++q) {
            ww[q] = nx[q];
            vm |= (off + q * WAVE + lane < rd ? 1u : 0u) << q;
          }
          const uint32_t nxt = off + NWAVES * PIECE;
          if (nxt < rd) {
#pragma unroll
            for (int q = 0; q < U; ++q) nx[q] = cl[rst + min(nxt + q * WAVE + lane, rd - 1)];
          }
          process(ww, vm, [&](int) -> uint32_t { return sl; });
        }
      }
    }

    // ---- short rows, window by window.  Every lane of a wave runs the same number of
    // windows because the ballots and shuffles must not see inactive lanes.
    for (uint32_t e0 = 0; e0 < tot; e0 += WIN) {
      const uint32_t kn = wk == 2 ? 0u : wk + 1;
      // clear every word: scans of other modes use more words of the same masks
      if (tid < (uint32_t)Lds<BLOCK>::MASK_WORDS) L.wmask[kn][tid] = 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (cls[q] == 1) {
          const uint32_t s0 = pos[q];
          if (s0 > e0 && s0 - e0 < WIN)
            atomicOr(&L.wmask[wk][(s0 - e0) >> 5], 1u << ((s0 - e0) & 31));
          if (s0 <= e0 && e0 - s0 < d[q]) L.wfirst[wk] = slot[q];
        }
      }
      __syncthreads();
      const uint32_t word = lane < NWORDS ? L.wmask[wk][lane] : 0u;
      const uint32_t jf = L.wfirst[wk];
      wk = kn;
      // starts in the words before this wave's first word: their popcounts (at most
      // 32, six bits) summed one bit plane at a time with ballots
      const uint32_t fw = wid * (2 * U);  // this wave's first word (below 64)
      const uint32_t pc = (uint32_t)__popc(word);
      const uint64_t before_fw = (1ull << fw) - 1ull;
      uint32_t base = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b)
        base += (uint32_t)__popcll(__ballot((pc >> b) & 1u) & before_fw) << b;
      const bool hi_half = lane >= 32;
      uint32_t ww[U], jj[(U + 1) / 2];  // owners, two 16-bit slots per word
      uint32_t vm = 0;  // bit q: group q's arc of this lane exists
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const uint32_t wi = fw + 2 * q;  // group q covers words wi and wi + 1
        const uint32_t w0 = __builtin_amdgcn_readlane(word, wi);
        const uint32_t w1 = __builtin_amdgcn_readlane(word, wi + 1);
        const uint32_t p0 = base, p1 = base + (uint32_t)__popc(w0);
        base = p1 + (uint32_t)__popc(w1);
        const uint32_t j = jf + (hi_half ? p1 : p0) + (uint32_t)__popc((hi_half ? w1 : w0) & below);
        if (q % 2 == 0) jj[q / 2] = j;
        else jj[q / 2] |= j << 16;
        vm |= (e0 + fw * 32 + q * WAVE + lane < tot ? 1u : 0u) << q;
      }
      auto owner = [&](int q) -> uint32_t { return (jj[q / 2] >> (16 * (q % 2))) & 0xFFFFu; };
      // Lanes past the end of the arc space re-read its last arc (their owner is the
      // last short row), so every lane loads and the LDS reads and the row loads of
      // all U groups go out back to back.
#pragma unroll
      for (int q = 0; q < U; ++q) ww[q] = L.c_off[owner(q)];
#pragma unroll
      for (int q = 0; q < U; ++q) ww[q] = cl[ww[q] + min(e0 + fw * 32 + q * WAVE + lane, tot - 1)];
      process(ww, vm, owner);
    }
    __syncthreads();
  }
}

// Ascending bitonic sort of up to 64 keys held one per lane (missing lanes hold ~0),
// in registers by one wave.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t k = 2; k <= (uint32_t)WAVE; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const uint64_t other = __shfl_xor(x, (int)j, WAVE);
      const bool up = (lane & k) == 0;
      const bool low = (lane & j) == 0;
      x = (low == up) ? (x < other ? x : other) : (x > other ? x : other);
    }
  }
  return x;
}

// In-place ascending bitonic sort of keys[0, M), M a power of two, by the workgroup.
template <int BLOCK>
__device__ void bitonic_sort(uint64_t *keys, uint32_t M) {
  for (uint32_t k = 2; k <= M; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < M; i += BLOCK) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = keys[i], b = keys[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// The same network over an array split in two LDS parts: element i is lo[i] below nlo,
// hi[i - nlo] above.
template <int BLOCK>
__device__ void bitonic_sort2(uint64_t *lo, uint32_t nlo, uint64_t *hi, uint32_t M) {
  auto at = [&](uint32_t i) -> uint64_t & { return i < nlo ? lo[i] : hi[i - nlo]; };
  for (uint32_t k = 2; k <= M; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < M; i += BLOCK) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = at(i), b = at(ixj);
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            at(i) = b;
            at(ixj) = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

constexpr uint32_t pow2floor(uint32_t x) { return x <= 1 ? 1u : 2u * pow2floor(x / 2); }

// One backtracking walk of a wave (section 4, "by backtracking"): from `start` on
// level `lev` of side `side` down to level 0.  Each step draws r < sigma(x) and takes,
// among x's neighbours on the level below in row order (the s side looks at
// predecessors in x's in-row, the t side at successors in x's out-row), the first
// whose running count exceeds r.  Rows are sorted, so "row order" is "ascending id".
// Two equivalent ways to enumerate those neighbours:
//   row scan  -- walk x's row, keep entries tagged with the level below;
//   list scan -- walk the (remembered) node list of the level below and keep the
//                entries found in x's row by binary search; prefix sums are then
//                taken in ascending id.  Used when the list is much shorter than the
//                row (x a hub).
// HASHED: records in a table of 2^hbits (see Recs), vh[j] the record index of visit[j].
template <bool HASHED>
__device__ void backtrack(const GraphDev &g, uint32_t side, uint32_t start, uint32_t lev,
                          uint32_t *rec, uint32_t hbits, const uint32_t *visit,
                          const uint32_t *vh,
                          const uint32_t (*seg_lo)[MAXLEV], const uint32_t (*seg_hi)[MAXLEV],
                          MatchScratch &M, uint64_t seed, uint64_t i, uint32_t phase,
                          uint32_t *path, uint32_t ls, uint32_t base, uint32_t endpoint,
                          uint32_t &flags) {
  const uint32_t lane = lane_id();
  const uint32_t *rp = side == 0 ? g.rrow : g.row;
  const uint32_t *cl = side == 0 ? g.rcol : g.col;
  const uint64_t lanes_below = (1ULL << lane) - 1ULL;
  const Recs R{rec, hbits};
  uint32_t x = start;
  for (uint32_t j = lev; j >= 1; --j) {
    // A level of one node holds x's only predecessor, whatever the draw (the draw is
    // skipped: every draw is a pure function of its counter, so no other draw moves).
    // Level 0 is the endpoint itself.
    if (j == 1 || (j - 1 < (uint32_t)MAXLEV && seg_hi[side][j - 1] - seg_lo[side][j - 1] == 1)) {
      x = j == 1 ? endpoint : visit[seg_lo[side][j - 1]];
      if (lane == 0) path[side == 0 ? j - 1 : ls + 1 + (lev - j) + 1] = x + base;
      continue;
    }
    const uint32_t beg = rp[x], end = rp[x + 1];  // in flight during the draw
    const u128 bound = node_sig<HASHED>(R, x, flags);
    const u128 r = uniform_below(bound, seed, i, stream_word(phase, side == 0 ? P_BACK_S : P_BACK_T, j),
                                 flags);
    const uint32_t want = (side == 0 ? 0u : TAG_T) | j;  // level j-1, stored as (j-1)+1
    uint32_t pick = 0xFFFFFFFFu;
    bool row_scan = true;
    if (j - 1 < (uint32_t)MAXLEV) {
      const uint32_t Lb = seg_lo[side][j - 1], Le = seg_hi[side][j - 1];
      if ((uint64_t)(Le - Lb) * 16 < (uint64_t)(end - beg)) {
        // ---- list scan
        uint32_t nm = 0;
        for (uint32_t b = Lb; b < Le; b += WAVE) {
          const uint32_t q = b + lane;
          uint32_t cand = 0;
          bool match = false;
          if (q < Le) {
            cand = visit[q];
            // the arc between cand and x (cand -> x on the s side, x -> cand on the t
            // side) is searched in the shorter of x's row and cand's row of the other
            // direction: x is usually a hub, cand usually not
            const uint32_t *orp = side == 0 ? g.row : g.rrow;
            const uint32_t *ocl = side == 0 ? g.col : g.rcol;
            const uint32_t cb = orp[cand], ce = orp[cand + 1];
            const bool in_cand = ce - cb < end - beg;
            const uint32_t *arr = in_cand ? ocl : cl;
            const uint32_t target = in_cand ? x : cand;
            uint32_t lo = in_cand ? cb : beg, hi = in_cand ? ce : end;
            const uint32_t stop = hi;
            while (lo < hi) {
              const uint32_t mid = (lo + hi) >> 1;
              if (arr[mid] < target) lo = mid + 1; else hi = mid;
            }
            match = lo < stop && arr[lo] == target;
          }
          const uint64_t mk = __ballot(match);
          if (match) {
            const uint32_t pos = nm + (uint32_t)__popcll(mk & lanes_below);
            if (pos < (uint32_t)MATCH_CAP) {
              const u128 sv = ld_sig(rec, HASHED ? vh[q] : cand);
              M.id[pos] = cand;
              M.lo[pos] = sv.lo;
              M.hi[pos] = sv.hi;
            }
          }
          nm += (uint32_t)__popcll(mk);
        }
        if (nm <= (uint32_t)MATCH_CAP) {
          row_scan = false;
          // inclusive prefix of match q in id order = sum of sigma over ids <= id_q
          uint32_t found = 0xFFFFFFFFu;
          for (uint32_t q0 = 0; q0 < nm; q0 += WAVE) {
            const uint32_t q = q0 + lane;
            if (q < nm) {
              const uint32_t me = M.id[q];
              u128 inc{0, 0};
              bool dm = false;
              for (uint32_t p2 = 0; p2 < nm; ++p2)
                if (M.id[p2] <= me) inc = add128(inc, u128{M.lo[p2], M.hi[p2]}, dm);
              const u128 exc = sub128(inc, u128{M.lo[q], M.hi[q]});
              if (!lt128(r, exc) && lt128(r, inc)) found = me;
            }
          }
          const uint64_t mk = __ballot(found != 0xFFFFFFFFu);
          if (mk) pick = __shfl(found, (int)__ffsll((unsigned long long)mk) - 1, WAVE);
        }
      }
    }
    if (row_scan) {
      u128 carry{0, 0};
      for (uint32_t b = beg; b < end; b += WAVE) {
        const uint32_t idx = b + lane;
        uint32_t u = 0;
        u128 val{0, 0};
        if (idx < end) {
          u = cl[idx];
          if (HASHED) {
            uint32_t h;
            const uint64_t xw = rec_find(R, u, h);
            if (h != NO_REC && (uint32_t)xw == want) val = ld_sig(rec, h);
          } else if (ld_tag(tag_of(rec, u)) == want) {
            val = ld_sig(rec, u);
          }
        }
        bool dummy = false;
        u128 inc = wave_incl_u128(val, dummy);
        inc = add128(inc, carry, dummy);
        const uint64_t m = __ballot(idx < end && lt128(r, inc));
        if (m) {
          pick = __shfl(u, (int)__ffsll((unsigned long long)m) - 1, WAVE);
          break;
        }
        carry.lo = __shfl(inc.lo, WAVE - 1, WAVE);
        carry.hi = __shfl(inc.hi, WAVE - 1, WAVE);
      }
    }
    if (pick == 0xFFFFFFFFu) {
      flags |= FLAG_CAPACITY;  // unreachable for consistent counts
      return;
    }
    x = pick;
    if (lane == 0) path[side == 0 ? j - 1 : ls + 1 + (lev - j) + 1] = x + base;
  }
}

// MULTI = false: one graph and seed, sample id first0 + k for launch index k.
// MULTI = true: launch index k belongs to the segment segs[j] with the largest
// begin <= k; graph, seed, phase and id come from there.
// A level expansion of at most small_exp arcs takes one combined scan; larger ones
// take a touch scan and, if the searches did not meet, a discovery scan.
// HASHED: the slots' records are tables of 2^st.hbits (see Recs) instead of one record
// per node.
// Occupancy targets: 5 waves per SIMD (VGPR-bound) for 128 and 256 threads; 64-thread
// workgroups are LDS-bound at 4.  With tables 4: the probes' state takes the registers
// that a fifth wave would leave (it would spill).
template <int BLOCK, bool MULTI, bool HASHED>
__global__ __launch_bounds__(BLOCK, (BLOCK == 64 || HASHED) ? 4 : 5) void sampler_kernel(GraphDev g0, SlotState st, uint64_t seed_a,
                                                        uint32_t phase_a, uint64_t first_a,
                                                        const SampleSeg *__restrict__ segs,
                                                        uint32_t nseg_a, uint32_t count_a,
                                                        uint32_t *work, SampleOut out_a,
                                                        uint32_t small_exp,
                                                        const BatchDesc *__restrict__ bd) {
  constexpr int NWAVES = BLOCK / WAVE;
  SampleOut out = out_a;
  if (bd && bd->stride) out.stride = bd->stride;
  // a replayed launch takes its batch from the descriptor (uniform, scalar loads)
  const uint64_t seed0 = bd ? bd->seed : seed_a, first0 = bd ? bd->first : first_a;
  const uint32_t phase0 = bd ? bd->phase : phase_a, count = bd ? bd->count : count_a;
  const uint32_t nseg = bd ? bd->nseg : nseg_a;
  __shared__ Lds<BLOCK> L;
  const uint32_t tid = threadIdx.x, wid = tid / WAVE, lane = lane_id();
  const size_t n = st.n;  // slot capacity
  const size_t slot = blockIdx.x;
  uint32_t *rec = st.rec + slot * n * REC_WORDS;
  uint32_t *visit = st.visit + slot * n;
  uint32_t *vh = HASHED ? st.vh + slot * n : nullptr;
  uint64_t *gpi = st.pi + slot * st.pi_cap;
  const uint32_t hbits = HASHED ? st.hbits : 0u;
  const Recs R{rec, hbits};

  for (uint32_t j = tid; j < (uint32_t)FILTER_WORDS; j += BLOCK) L.filter[j] = 0;
  for (uint32_t j = tid; j < 3u * Lds<BLOCK>::MASK_WORDS; j += BLOCK) (&L.wmask[0][0])[j] = 0;
  uint32_t wk = 0;  // arc-window counter of scan_frontier (mod 3)

  // Sample ids: the first three quarters of the rounds are dealt out statically
  // (workgroup b takes b, b + grid, ...); the rest come from the shared counter, which
  // evens out the tail.  A device-wide atomic is a slow round trip, so tid 0 fetches
  // the next id while the current sample starts.
  const uint32_t grid = gridDim.x;
  const uint32_t rounds = count / grid - (count / grid) / 4;
  const uint32_t static_end = rounds * grid;
  uint32_t taken = 0;  // static ids taken by this workgroup (tid 0)
  auto next_id = [&]() -> uint32_t {
    if (taken < rounds) return blockIdx.x + grid * taken++;
    return static_end + atomicAdd(work, 1u);
  };
  uint32_t k_next = tid == 0 ? next_id() : 0u;
  for (;;) {
    if (tid == 0) {
      const uint32_t k = k_next;
      L.k = k;
      if (MULTI && k < count) {
        uint32_t lo = 0, hi = nseg;  // largest j with segs[j].begin <= k
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (segs[mid].begin <= k) lo = mid; else hi = mid;
        }
        L.seg = lo;
      }
    }
    __syncthreads();
    const uint32_t k = L.k;
    if (k >= count) break;
    GraphDev g = g0;
    uint64_t seed = seed0, i = first0 + k;
    uint32_t phase = phase0, base = 0;
    if (MULTI) {
      const SampleSeg &S = segs[__builtin_amdgcn_readfirstlane(L.seg)];
      g.n = S.n;
      g.row = S.row;
      g.col = S.col;
      g.rrow = S.rrow;
      g.rcol = S.rcol;
      g.forward = S.forward;
      seed = S.seed;
      phase = S.phase;
      i = S.first + (k - S.begin);
      base = S.id_base;
      if (S.wide_only) {  // left to the wide-count kernel (uniform for the workgroup)
        if (tid == 0) {
          k_next = next_id();
          out.flags[k] = FLAG_OVERFLOW;
          out.len[k] = 0;
          if (out.fix_list) out.fix_list[atomicAdd(out.fix_count, 1u)] = k;
        }
        __syncthreads();  // every thread has read L.k and L.seg before they change
        continue;
      }
    }

    // ---- the pair and the two initial levels (lanes 0 and 1 draw s and t' side by side)
    if (wid == 0) {
      uint32_t fl = 0, x = 0;
      if (lane < 2)
        x = (uint32_t)uniform_below(u128{lane == 0 ? g.n : g.n - 1u, 0}, seed, i,
                                    stream_word(phase, lane == 0 ? P_S : P_T, 0), fl).lo;
      const uint32_t s = __builtin_amdgcn_readlane(x, 0);
      const uint32_t tp = __builtin_amdgcn_readlane(x, 1);
      fl = __builtin_amdgcn_readlane(fl, 0) | __builtin_amdgcn_readlane(fl, 1);
      if (lane == 0) {
      k_next = next_id();
      const uint32_t t = tp + (tp >= s ? 1u : 0u);
      L.s = s;
      L.t = t;
      // the table is empty: s takes its home record, t its own or the next one
      const uint32_t hs = HASHED ? R.home(s) : s;
      const uint32_t ht = HASHED ? (R.home(t) == hs ? (hs + 1u) & R.mask() : R.home(t)) : t;
      *tag_of(rec, hs) = 1u;
      *tag_of(rec, ht) = TAG_T | 1u;
      if (HASHED) {
        *pos_of(rec, hs) = s + 1u;
        *pos_of(rec, ht) = t + 1u;
        vh[0] = hs;
        vh[1] = ht;
      }
      sig_of(rec, hs)[0] = 1;
      sig_of(rec, hs)[1] = 0;
      sig_of(rec, ht)[0] = 1;
      sig_of(rec, ht)[1] = 0;
      visit[0] = s;
      visit[1] = t;
      L.fb[0] = 0; L.fe[0] = 1;
      L.fb[1] = 1; L.fe[1] = 2;
      L.seg_lo[0][0] = 0; L.seg_hi[0][0] = 1;
      L.seg_lo[1][0] = 1; L.seg_hi[1][0] = 2;
      L.lvl[0] = 0; L.lvl[1] = 0;
      const uint32_t s0 = g.row[s], t0 = g.rrow[t];
      L.st0[0] = s0;
      L.st0[1] = t0;
      L.deg[0] = (uint64_t)(g.row[s + 1] - s0);
      L.deg[1] = (uint64_t)(g.rrow[t + 1] - t0);
      L.arcs = 0;
      L.nvis = 2;
      L.flags = fl;
      L.ovf_any = 0;
      }
    }
    __syncthreads();

    bool ovf = false;
    bool met = false;
    uint32_t needed = 0;
    for (;;) {
      // a head found no room in the table: the wide-count kernel samples this pair
      if (HASHED && (L.flags & FLAG_CAPACITY)) break;
      // ties expand the s side; the forward search expands it always
      const uint32_t me = (g.forward || L.deg[0] <= L.deg[1]) ? 0u : 1u;
      const uint32_t ot = 1u - me;
      const uint32_t fb = L.fb[me], fe = L.fe[me];
      const uint32_t ob = L.fb[ot], oe = L.fe[ot];
      const uint32_t lme = L.lvl[me], lot = L.lvl[ot];
      const uint32_t other_tag = (ot == 0 ? 0u : TAG_T) | (lot + 1);
      const uint32_t next_tag = (me == 0 ? 0u : TAG_T) | (lme + 2);
      const uint64_t dme = L.deg[me];
      // (tid 0 resets fields read only before the previous level's last barrier; the
      // barrier before each scan publishes the resets)
      if (tid == 0) {
        L.arcs += dme;
        L.pi_count = 0;
        L.new_deg = 0;
      }
      const uint32_t nb = L.nvis;  // the next level starts here
      needed = nb;
      if (dme <= (uint64_t)small_exp) {
        // small level: meeting test by tag and discovery in one pass (the nodes it
        // claims are never read if the two searches touched; they are reset anyway)
        __syncthreads();
        bool ovf_next = false;  // counts of the next level matter only if there is one
        scan_frontier<BLOCK, Scan::Both, HASHED>(L, g, me, fb, fe, rec, hbits, visit, vh, gpi,
                                                 st.pi_cap, other_tag, next_tag, ovf_next, wk,
                                                 false, lme == 0);
        if (L.pi_count > 0) {
          met = true;
          break;
        }
        ovf |= ovf_next;
      } else {
        // the other side's frontier: a bit filter, and an exact set when it is small
        constexpr uint32_t FSET_SLOTS = 4 * Lds<BLOCK>::CHUNK;
        const bool exact = oe - ob <= FSET_SLOTS / 2;
        if (exact) {
          for (uint32_t j = tid; j < FSET_SLOTS; j += BLOCK) L.fset[j] = FSET_EMPTY;
          __syncthreads();
        }
        for (uint32_t j = ob + tid; j < oe; j += BLOCK) {
          const uint32_t v = visit[j];
          const uint32_t h = filter_bit(v);
          atomicOr(&L.filter[h >> 5], 1u << (h & 31));
          if (exact) fset_insert<FSET_SLOTS>(L.fset, v);
        }
        __syncthreads();
        scan_frontier<BLOCK, Scan::Touch, HASHED>(L, g, me, fb, fe, rec, hbits, visit, vh, gpi,
                                                  st.pi_cap, other_tag, next_tag, ovf, wk, exact,
                                                  lme == 0, ob, oe - ob);
        for (uint32_t j = tid; j < (uint32_t)FILTER_WORDS; j += BLOCK) L.filter[j] = 0;
        const uint32_t P = L.pi_count;  // final: the scan ends with a barrier
        if (P > 0) {
          met = true;
          break;
        }
        scan_frontier<BLOCK, Scan::Discover, HASHED>(L, g, me, fb, fe, rec, hbits, visit, vh,
                                                     gpi, st.pi_cap, other_tag, next_tag, ovf,
                                                     wk, false, lme == 0);
      }
      // final: every scan ends with a barrier; tid 0 writes other fields below
      const uint32_t ne = L.nvis;
      const uint64_t nd = L.new_deg;
      if (ne == nb) break;  // the expanded side closed: s and t are disconnected
      if (tid == 0) {
        L.fb[me] = nb;
        L.fe[me] = ne;
        L.lvl[me] = lme + 1;
        L.deg[me] = nd;
        if (lme + 1 < (uint32_t)MAXLEV) {
          L.seg_lo[me][lme + 1] = nb;
          L.seg_hi[me][lme + 1] = ne;
        }
      }
      __syncthreads();
    }
    if (ovf) atomicOr(&L.ovf_any, 1u);
    __syncthreads();
    if (tid == 0) L.needed = needed;
    if (L.ovf_any && tid == 0) L.flags |= FLAG_OVERFLOW;
    __syncthreads();

    const uint32_t ls = L.lvl[0], lt = L.lvl[1];
    uint32_t len = 0;
    uint32_t *path = out.path + (size_t)k * out.stride;
    if (met && L.flags == 0) {
      const uint32_t P = L.pi_count;
      if (P > st.pi_cap || ls + lt + 2 > out.stride) {
        if (tid == 0) L.flags |= FLAG_CAPACITY;
      } else {
        // ---- candidate edges in canonical order (v ascending, then w ascending), weight
        // sigma_s(v) sigma_t(w) each; draw r < sigma_st = the sum of the weights and
        // take the edge whose interval of prefixes holds r
        bool arena = false;  // the sort used the filter's words (cleared again below)
        if (P <= (uint32_t)BLOCK) {
          // one candidate per thread, no sort: a candidate's prefix in canonical order is
          // the sum of the weights of the smaller keys (keys are distinct).  Each thread
          // sums every weight itself and takes the draw itself (a pure function of the
          // sample), so one barrier publishes the weights and the one after the pick its
          // winner.
          bool wov = false;
          uint64_t key = 0;
          u128 wt{0, 0};
          if (tid < P) {
            key = L.pi[tid];
            if (HASHED) {
              uint32_t nfl = 0;  // an endpoint without a record (never, for consistent tables)
              wt = mul128(node_sig<true>(R, (uint32_t)(key >> 32), nfl),
                          node_sig<true>(R, (uint32_t)key, nfl), wov);
              if (nfl) atomicOr(&L.flags, nfl);
            } else {
              wt = mul128(ld_sig(rec, (uint32_t)(key >> 32)), ld_sig(rec, (uint32_t)key), wov);
            }
            L.c_sig_lo[tid] = wt.lo;
            L.c_sig_hi[tid] = wt.hi;
            if (wov) atomicOr(&L.ovf_any, 2u);
          }
          if (tid == 0) {
            L.win = 0xFFFFFFFFu;
            L.wkey = L.pi[0];
          }
          __syncthreads();
          if (tid < P) {
            u128 pre{0, 0}, total{0, 0};
            bool dm = false, tov = false;  // a total that fits has partial sums that fit
#pragma unroll 4
            for (uint32_t j = 0; j < P; ++j) {
              const u128 x{L.c_sig_lo[j], L.c_sig_hi[j]};
              if (L.pi[j] < key) pre = add128(pre, x, dm);
              total = add128(total, x, tov);
            }
            uint32_t fl = (tov || (L.ovf_any & 2u)) ? (uint32_t)FLAG_OVERFLOW : 0u;
            if (fl == 0) {
              const u128 r = uniform_below(total, seed, i, stream_word(phase, P_EDGE, 0), fl);
              if (fl == 0 && !lt128(r, pre) && lt128(r, add128(pre, wt, dm))) {
                L.win = tid;
                L.wkey = key;
              }
            }
            if (tid == 0) L.flags |= fl;  // every thread found the same flags
          }
        } else {
          // sort, then prefix sums chunk by chunk.  Up to SORT_CAP keys are sorted in the
          // LDS words the searches no longer need, more in the slot's candidate buffer.
          constexpr uint32_t NLO = FILTER_WORDS / 2, NHI = 2 * Lds<BLOCK>::CHUNK;
          constexpr uint32_t SORT_CAP = pow2floor(NLO + NHI);
          uint32_t M = 1;
          while (M < P) M <<= 1;
          arena = M <= SORT_CAP;
          if (arena) {
            for (uint32_t j = tid; j < M; j += BLOCK) {
              const uint64_t x = j < P ? (j < (uint32_t)PI_LDS ? L.pi[j] : gpi[j]) : ~0ULL;
              if (j < NLO) L.sort_lo[j] = x;
              else L.sort_hi[j - NLO] = x;
            }
            __syncthreads();
            bitonic_sort2<BLOCK>(L.sort_lo, NLO, L.sort_hi, M);
          } else {
            for (uint32_t j = tid; j < (uint32_t)PI_LDS; j += BLOCK) gpi[j] = L.pi[j];
            for (uint32_t j = P + tid; j < M; j += BLOCK) gpi[j] = ~0ULL;
            __syncthreads();
            bitonic_sort<BLOCK>(gpi, M);
          }
          auto key_at = [&](uint32_t j) -> uint64_t {
            return arena ? (j < NLO ? L.sort_lo[j] : L.sort_hi[j - NLO]) : gpi[j];
          };
          bool wov = false;
          u128 acc{0, 0};
          if (HASHED) {
            uint32_t nfl = 0;  // an endpoint without a record (never, for consistent tables)
            for (uint32_t j = tid; j < P; j += BLOCK) {
              const uint64_t key = key_at(j);
              acc = add128(acc, mul128(node_sig<true>(R, (uint32_t)(key >> 32), nfl),
                                       node_sig<true>(R, (uint32_t)key, nfl), wov), wov);
            }
            if (nfl) atomicOr(&L.flags, nfl);
          } else {
            for (uint32_t j = tid; j < P; j += BLOCK) {
              const uint64_t key = key_at(j);
              acc = add128(acc, mul128(ld_sig(rec, (uint32_t)(key >> 32)), ld_sig(rec, (uint32_t)key), wov), wov);
            }
          }
          u128 total;
          (void)block_incl_u128(L, acc, total, wov);
          if (wov) atomicOr(&L.ovf_any, 2u);
          __syncthreads();
          if (tid == 0) {
            if (L.ovf_any & 2u) {
              L.flags |= FLAG_OVERFLOW;
            } else {
              uint32_t fl = 0;
              const u128 r = uniform_below(total, seed, i, stream_word(phase, P_EDGE, 0), fl);
              L.flags |= fl;
              L.r_lo = r.lo;
              L.r_hi = r.hi;
            }
            L.win = 0xFFFFFFFFu;
            L.wkey = key_at(0);
          }
          __syncthreads();
          if (L.flags == 0) {
            const u128 r{L.r_lo, L.r_hi};
            u128 carry{0, 0};
            for (uint32_t c0 = 0; c0 < P; c0 += BLOCK) {
              const uint32_t j = c0 + tid;
              u128 wt{0, 0};
              bool dm = false;
              uint64_t key = 0;
              if (j < P) {
                key = key_at(j);
                if (HASHED) {
                  uint32_t nfl = 0;  // checked by the first pass over the same keys
                  wt = mul128(node_sig<true>(R, (uint32_t)(key >> 32), nfl),
                              node_sig<true>(R, (uint32_t)key, nfl), dm);
                } else {
                  wt = mul128(ld_sig(rec, (uint32_t)(key >> 32)), ld_sig(rec, (uint32_t)key), dm);
                }
              }
              u128 chunk_total;
              u128 inc = block_incl_u128(L, wt, chunk_total, dm);
              inc = add128(inc, carry, dm);
              const u128 exc = sub128(inc, wt);
              if (j < P && !lt128(r, exc) && lt128(r, inc)) {
                L.win = j;
                L.wkey = key;
              }
              carry = add128(carry, chunk_total, dm);
            }
          }
        }
        __syncthreads();
        if (arena)  // the filter is all zero between searches
          for (uint32_t j = tid; j < (uint32_t)FILTER_WORDS; j += BLOCK) L.filter[j] = 0;
        if (L.flags == 0) {
          const uint32_t win = L.win;
          const uint64_t key = L.wkey;  // a candidate of this sample even if none was won
          const uint32_t v = (uint32_t)(key >> 32), w = (uint32_t)key;
          __syncthreads();  // the staging area becomes backtracking scratch below
          // ---- the two halves: with two or more waves, wave 0 walks to s while wave 1
          // walks to t; a single wave walks one after the other
          uint32_t fl = 0;
          MatchScratch *mscr = reinterpret_cast<MatchScratch *>(L.pi);
          if (wid == 0) {
            if (lane == 0) path[ls] = v + base;
            backtrack<HASHED>(g, 0, v, ls, rec, hbits, visit, vh, L.seg_lo, L.seg_hi, mscr[0],
                              seed, i, phase, path, ls, base, L.s, fl);
          }
          if (wid == (NWAVES >= 2 ? 1u : 0u)) {
            if (lane == 0) path[ls + 1] = w + base;
            backtrack<HASHED>(g, 1, w, lt, rec, hbits, visit, vh, L.seg_lo, L.seg_hi, mscr[1],
                              seed, i, phase, path, ls, base, L.t, fl);
          }
          if (win >= P) fl |= FLAG_CAPACITY;
          if (fl && lane == 0) atomicOr(&L.flags, fl);
          __syncthreads();
          if (L.flags == 0) len = ls + lt + 2;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      out.s[k] = L.s;
      out.t[k] = L.t;
      out.len[k] = L.flags ? 0u : len;
      out.arcs[k] = L.arcs;
      out.flags[k] = L.flags;
      out.nodes[k] = L.needed;
      // counts beyond 128 bits, or more candidate edges than the slot holds: sampled again
      // by the wide-count kernel, which has neither limit
      if ((L.flags & (FLAG_OVERFLOW | FLAG_CAPACITY)) && out.fix_list)
        out.fix_list[atomicAdd(out.fix_count, 1u)] = k;
    }
    // ---- restore the slot's all-zero state for the next sample
    const uint32_t nv = L.nvis;
    for (uint32_t j = tid; j < nv; j += BLOCK) {
      uint4 *r4 = reinterpret_cast<uint4 *>(tag_of(rec, HASHED ? vh[j] : visit[j]));
      r4[0] = make_uint4(0, 0, 0, 0);  // tag, position, count low
      r4[1] = make_uint4(0, 0, 0, 0);  // count high (and the unused words)
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ hit reduction
// Two passes per check interval.  partition: each workgroup takes a slice of the
// samples, counts its interior hits per node tile in LDS, reserves room in each
// tile's bin with one atomic per (workgroup, tile) and copies the hits there.  tile:
// one workgroup per tile builds an LDS histogram of its bin and adds it to the
// counters of the tile -- every counter has a single owner, so the counters see no
// atomics.
constexpr int HIT_BLOCK = 256;
constexpr uint32_t HIT_TILE = 8192;   // node ids per tile (32 KB LDS histogram)
constexpr uint32_t SAMPLES_PER_PART = 64;

// Bin entries pack a node id (below 2^25) with a multiplicity (at most the samples of
// one partition workgroup) in the top 7 bits.
constexpr uint32_t ENTRY_ID_BITS = 25;
constexpr uint32_t AGG_SLOTS = 1024;  // LDS hash of one partition workgroup's hits
static_assert(SAMPLES_PER_PART < (1u << (32 - ENTRY_ID_BITS)), "multiplicity fits its bits");
static_assert(AGG_SLOTS == 1024, "the probe hash takes 10 bits");
static_assert((uint64_t)MAX_HIT_TILES * HIT_TILE <= (1ull << ENTRY_ID_BITS), "ids fit their bits");

// spp samples per workgroup.  With aggregate, spp * (stride - 2) <= AGG_SLOTS / 2, so
// the LDS hash is at most half full and every probe sequence ends; without it (paths
// too long for the hash) every hit is its own entry of multiplicity 1.
// pass: PASS_FIXED reserves room in fixed-size bins and writes the entries;
// PASS_COUNT only adds the workgroup's entries per tile to bin_count; PASS_WRITE
// writes them at tile_start[t] + (a place reserved through tile_fill[t]).
enum : int { PASS_FIXED = 0, PASS_COUNT = 1, PASS_WRITE = 2 };

__global__ __launch_bounds__(HIT_BLOCK) void hit_partition_kernel(
    const uint32_t *path, const uint32_t *len, uint32_t stride, uint32_t nsamp, uint32_t tiles,
    uint32_t spp, int aggregate, int pass, uint32_t *bins, uint64_t cap, uint32_t *bin_count,
    const uint32_t *tile_start, uint32_t *tile_fill) {
  __shared__ uint32_t tcount[MAX_HIT_TILES];
  __shared__ uint32_t tbase[MAX_HIT_TILES];
  __shared__ uint32_t akey[AGG_SLOTS];
  __shared__ uint32_t acnt[AGG_SLOTS];
  const uint32_t s0 = blockIdx.x * spp;
  const uint32_t s1 = min(nsamp, s0 + spp);
  const uint32_t entries = (s1 - s0) * stride;
  for (uint32_t t = threadIdx.x; t < tiles; t += HIT_BLOCK) tcount[t] = 0;
  // reserve room for this workgroup's tcount[t] entries of every tile
  auto reserve = [&]() {
    for (uint32_t t = threadIdx.x; t < tiles; t += HIT_BLOCK) {
      const uint32_t c = tcount[t];
      if (c) {
        if (pass == PASS_FIXED) tbase[t] = atomicAdd(&bin_count[t], c);
        else if (pass == PASS_COUNT) atomicAdd(&bin_count[t], c);
        else tbase[t] = tile_start[t] + atomicAdd(&tile_fill[t], c);
      }
      tcount[t] = 0;
    }
  };
  auto slot_of = [&](uint32_t t, uint32_t pos) -> size_t {
    return pass == PASS_FIXED ? (size_t)t * cap + pos : (size_t)pos;
  };
  if (!aggregate) {
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < entries; e += HIT_BLOCK) {
      const uint32_t k = s0 + e / stride, j = e % stride;
      if (j >= 1 && j + 1 < len[k]) atomicAdd(&tcount[path[(size_t)k * stride + j] / HIT_TILE], 1u);
    }
    __syncthreads();
    reserve();
    if (pass == PASS_COUNT) return;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < entries; e += HIT_BLOCK) {
      const uint32_t k = s0 + e / stride, j = e % stride;
      if (j >= 1 && j + 1 < len[k]) {
        const uint32_t v = path[(size_t)k * stride + j];
        const uint32_t t = v / HIT_TILE;
        const uint32_t pos = tbase[t] + atomicAdd(&tcount[t], 1u);
        bins[slot_of(t, pos)] = v | (1u << ENTRY_ID_BITS);
      }
    }
    return;
  }
  for (uint32_t q = threadIdx.x; q < AGG_SLOTS; q += HIT_BLOCK) {
    akey[q] = 0xFFFFFFFFu;
    acnt[q] = 0;
  }
  __syncthreads();
  // aggregate the slice's interior hits by node (a hub appears on many paths)
  for (uint32_t e = threadIdx.x; e < entries; e += HIT_BLOCK) {
    const uint32_t k = s0 + e / stride, j = e % stride;
    if (j >= 1 && j + 1 < len[k]) {
      const uint32_t v = path[(size_t)k * stride + j];
      uint32_t h = (v * 2654435761u) >> 22;  // 10 bits
      for (;;) {  // at most AGG_SLOTS / 2 keys: a free slot is always found
        const uint32_t old = atomicCAS(&akey[h], 0xFFFFFFFFu, v);
        if (old == 0xFFFFFFFFu || old == v) break;
        h = (h + 1) & (AGG_SLOTS - 1);
      }
      atomicAdd(&acnt[h], 1u);
    }
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < AGG_SLOTS; q += HIT_BLOCK)
    if (acnt[q]) atomicAdd(&tcount[akey[q] / HIT_TILE], 1u);
  __syncthreads();
  reserve();
  if (pass == PASS_COUNT) return;
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < AGG_SLOTS; q += HIT_BLOCK) {
    const uint32_t c = acnt[q];
    if (c) {
      const uint32_t v = akey[q];
      const uint32_t t = v / HIT_TILE;
      const uint32_t pos = tbase[t] + atomicAdd(&tcount[t], 1u);
      bins[slot_of(t, pos)] = v | (c << ENTRY_ID_BITS);  // in range (see the launcher)
    }
  }
}

// Exclusive prefix sum of bin_count[0, tiles) into tile_start (one workgroup).
static_assert(MAX_HIT_TILES % HIT_BLOCK == 0, "tiles split evenly over the scan's threads");
__global__ __launch_bounds__(HIT_BLOCK) void hit_scan_kernel(const uint32_t *bin_count,
                                                             uint32_t tiles,
                                                             uint32_t *tile_start) {
  __shared__ uint32_t part[HIT_BLOCK];
  constexpr uint32_t PER = MAX_HIT_TILES / HIT_BLOCK;
  const uint32_t b = threadIdx.x * PER;
  uint32_t sum = 0;
  for (uint32_t q = 0; q < PER; ++q)
    if (b + q < tiles) sum += bin_count[b + q];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < HIT_BLOCK; d <<= 1) {  // Hillis-Steele inclusive scan
    const uint32_t x = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (uint32_t q = 0; q < PER; ++q)
    if (b + q < tiles) {
      tile_start[b + q] = run;
      run += bin_count[b + q];
    }
}

// One workgroup per tile: LDS histogram of the tile's entries, then each node's
// counter is updated by the one thread that claims its histogram cell.
__global__ __launch_bounds__(HIT_BLOCK) void hit_tile_kernel(const uint32_t *bins, uint64_t cap,
                                                             uint32_t *bin_count,
                                                             const uint32_t *tile_start,
                                                             uint32_t *tile_fill, uint32_t n,
                                                             uint64_t *count, int subtract,
                                                             const uint32_t *group,
                                                             uint64_t *gmax) {
  __shared__ uint32_t hist[HIT_TILE];
  const uint32_t t = blockIdx.x;
  const uint32_t m = bin_count[t];
  if (m == 0) return;  // uniform for the workgroup
  const uint32_t tile0 = t * HIT_TILE;
  const uint32_t *bin = bins + (tile_start ? (size_t)tile_start[t] : (size_t)t * cap);
  constexpr uint32_t ID_MASK = (1u << ENTRY_ID_BITS) - 1u;
  for (uint32_t b = threadIdx.x; b < HIT_TILE; b += HIT_BLOCK) hist[b] = 0;
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < m; q += HIT_BLOCK) {
    const uint32_t x = bin[q];
    atomicAdd(&hist[(x & ID_MASK) - tile0], x >> ENTRY_ID_BITS);
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < m; q += HIT_BLOCK) {
    const uint32_t v = bin[q] & ID_MASK;
    const uint32_t h = atomicExch(&hist[v - tile0], 0u);  // the first claimer owns node v
    if (h && v < n) {
      const uint64_t c = subtract ? count[v] - h : count[v] + h;
      count[v] = c;
      // running maximum of the counts of each stopping-rule group (counts only grow
      // while the maxima are in use)
      if (gmax) {
        // most nodes of a popular group stay below its maximum: skip those atomics (a
        // stale read only costs an unneeded atomic)
        unsigned long long *gm = (unsigned long long *)&gmax[group[v]];
        if (c > __hip_atomic_load(gm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          atomicMax(gm, (unsigned long long)c);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // ready for the next call
    bin_count[t] = 0;
    if (tile_fill) tile_fill[t] = 0;
  }
}

// Histogram of pilot counts over [0, bins): the first LDS_BINS bins (where nearly every
// node falls) are aggregated per workgroup in LDS, higher counts go to global atomics.
// Counts never exceed bins - 1 (a pilot count is at most the pilot's sample count); the
// clamp only keeps every access in bounds.
constexpr uint32_t HIST_LDS_BINS = 4096;
__global__ __launch_bounds__(256) void count_hist_kernel(const uint64_t *__restrict__ count,
                                                         uint32_t n, uint32_t *hist,
                                                         uint32_t bins) {
  __shared__ uint32_t h[HIST_LDS_BINS];
  const uint32_t lb = min(bins, HIST_LDS_BINS);
  for (uint32_t j = threadIdx.x; j < lb; j += 256) h[j] = 0;
  __syncthreads();
  for (uint32_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
    const uint64_t c = count[v];
    const uint32_t b = c < bins ? (uint32_t)c : bins - 1;
    if (b < lb) atomicAdd(&h[b], 1u);
    else atomicAdd(&hist[b], 1u);
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < lb; j += 256)
    if (h[j]) atomicAdd(&hist[j], h[j]);
}

// group[v] = cgrp[pilot count of v]
__global__ __launch_bounds__(256) void group_map_kernel(const uint64_t *__restrict__ count,
                                                        uint32_t n,
                                                        const uint32_t *__restrict__ cgrp,
                                                        uint32_t bins, uint32_t *group) {
  for (uint32_t v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
    const uint64_t c = count[v];
    group[v] = cgrp[c < bins ? c : bins - 1];
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t count, uint32_t value) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = value;
}

// A copy by a kernel between device memory and pinned, coherent host memory (the GPU
// reads or writes the host side over the bus); the stream's next event covers it.
template <typename T>
__global__ __launch_bounds__(256) void copy_kernel(T *dst, const T *src, uint64_t count_a,
                                                   const BatchDesc *__restrict__ bd,
                                                   uint32_t per, uint32_t by_nseg) {
  const uint64_t count = bd ? (uint64_t)(by_nseg ? bd->nseg : bd->count) * per : count_a;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    dst[i] = src[i];
}

__global__ __launch_bounds__(256) void gather_kernel(const GatherDesc *__restrict__ d, uint32_t nd,
                                                     uint64_t *count_pool,
                                                     const uint64_t *gmax_pool, uint64_t *snap) {
  uint32_t lo = 0, hi = nd;  // descriptor with the largest block0 <= blockIdx.x
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (d[mid].block0 <= blockIdx.x) lo = mid; else hi = mid;
  }
  const GatherDesc g = d[lo];
  const uint64_t b = (uint64_t)(blockIdx.x - g.block0) * GATHER_CHUNK;
  const uint64_t e = min((uint64_t)g.len, b + GATHER_CHUNK);
  for (uint64_t j = b + threadIdx.x; j < e; j += 256) {
    if (g.mode == GATHER_GMAX) {
      snap[g.dst + j] = gmax_pool[g.off + j];
    } else {
      snap[g.dst + j] = count_pool[g.off + j];
      if (g.mode == GATHER_COUNT_ZERO) count_pool[g.off + j] = 0;
    }
  }
}

// ------------------------------------------------------------------ wide path counts
// wide_kernel: a sample whose 128-bit path counts overflowed is sampled again with
// multi-limb counts.  The procedure is the one of sampler_kernel (same pair, same
// level order, same draws; uniform_below consumes the same words whatever the width),
// so the result is the one exact arithmetic gives.  One workgroup per sample, working
// in a sampler slot's node records and node list (all zero between samples); the counts
// of level l of a side are stored contiguously, `stride` limbs per node in the order
// of the node list, with stride = (width of level l-1) + 1, which always holds the
// sum of the predecessors' counts; the level's width is then the widest count.
// A level is expanded in one arc-parallel pass: the thread that claims a new node
// pulls its count from the node's predecessors on the (complete) level before, so no
// two threads write the same count.
constexpr int WB = 512;
constexpr int WNW = WB / WAVE;

// Limb arrays: 64-bit limbs, least significant first.
__device__ uint32_t wide_len(const uint64_t *a, uint32_t w) {
  while (w > 0 && a[w - 1] == 0) --w;
  return w;
}

__device__ int wide_cmp(const uint64_t *a, uint32_t aw, const uint64_t *b, uint32_t bw) {
  aw = wide_len(a, aw);
  bw = wide_len(b, bw);
  if (aw != bw) return aw < bw ? -1 : 1;
  for (uint32_t j = aw; j-- > 0;)
    if (a[j] != b[j]) return a[j] < b[j] ? -1 : 1;
  return 0;
}

// The same for a number whose limb j sits at a[j * pitch] (a level's counts are stored
// limb-major: limb j of every node of the level side by side).
__device__ uint32_t wide_len_s(const uint64_t *a, uint32_t pitch, uint32_t w) {
  while (w > 0 && a[(size_t)(w - 1) * pitch] == 0) --w;
  return w;
}

// acc[0, aw) += x[j * pitch], j < xw, xw <= aw (x limb-major, acc contiguous).
__device__ void wide_add_s(uint64_t *acc, uint32_t aw, const uint64_t *x, uint32_t pitch,
                           uint32_t xw) {
  uint64_t c = 0;
  for (uint32_t j = 0; j < aw; ++j) {
    if (j >= xw && c == 0) break;
    const uint64_t xv = j < xw ? x[(size_t)j * pitch] : 0;
    const uint64_t s1 = acc[j] + xv;
    const uint64_t c1 = s1 < xv ? 1u : 0u;
    const uint64_t s2 = s1 + c;
    const uint64_t c2 = s2 < c ? 1u : 0u;
    acc[j] = s2;
    c = c1 | c2;
  }
}

// acc[0, aw) += x[0, xw), xw <= aw; returns the carry out of acc[aw - 1].
__device__ uint64_t wide_add(uint64_t *acc, uint32_t aw, const uint64_t *x, uint32_t xw) {
  uint64_t c = 0;
  for (uint32_t j = 0; j < aw; ++j) {
    if (j >= xw && c == 0) break;
    const uint64_t xv = j < xw ? x[j] : 0;
    const uint64_t s1 = acc[j] + xv;
    const uint64_t c1 = s1 < xv ? 1u : 0u;
    const uint64_t s2 = s1 + c;
    const uint64_t c2 = s2 < c ? 1u : 0u;
    acc[j] = s2;
    c = c1 | c2;
  }
  return c;
}

// out[0, aw + bw) = a * b (schoolbook), a and b limb-major with pitches ap and bp.
__device__ void wide_mul_s(const uint64_t *a, uint32_t ap, uint32_t aw, const uint64_t *b,
                           uint32_t bp, uint32_t bw, uint64_t *out) {
  for (uint32_t j = 0; j < aw + bw; ++j) out[j] = 0;
  for (uint32_t x = 0; x < aw; ++x) {
    const uint64_t ax = a[(size_t)x * ap];
    if (ax == 0) continue;
    uint64_t carry = 0;
    for (uint32_t y = 0; y < bw; ++y) {
      const uint64_t by = b[(size_t)y * bp];
      const uint64_t lo = ax * by, hi = __umul64hi(ax, by);
      uint64_t s = out[x + y] + lo;
      uint64_t c = s < lo ? 1u : 0u;
      s += carry;
      c += s < carry ? 1u : 0u;
      out[x + y] = s;
      carry = hi + c;  // the 128-bit sum fits, so this does not wrap
    }
    out[x + bw] = carry;
  }
}

// out[0, aw + bw) = a * b (schoolbook).
__device__ void wide_mul(const uint64_t *a, uint32_t aw, const uint64_t *b, uint32_t bw,
                         uint64_t *out) {
  for (uint32_t j = 0; j < aw + bw; ++j) out[j] = 0;
  for (uint32_t x = 0; x < aw; ++x) {
    const uint64_t ax = a[x];
    if (ax == 0) continue;
    uint64_t carry = 0;
    for (uint32_t y = 0; y < bw; ++y) {
      const uint64_t lo = ax * b[y], hi = __umul64hi(ax, b[y]);
      uint64_t s = out[x + y] + lo;
      uint64_t c = s < lo ? 1u : 0u;
      s += carry;
      c += s < carry ? 1u : 0u;
      out[x + y] = s;
      carry = hi + c;  // the 128-bit sum fits, so this does not wrap
    }
    out[x + bw] = carry;
  }
}

// r[0, bw) uniform in [0, bound), bound = bound[0, bw) >= 1, by the rule of
// uniform_below (W = bitlength(bound - 1), ceil(W/64) words per attempt taken from
// blocks 0, 1, ... of the attempt's counter, least-significant first).  tmp: bw limbs.
__device__ void uniform_below_wide(const uint64_t *bound, uint32_t bw, uint64_t seed, uint64_t i,
                                   uint64_t sword, uint64_t *r, uint64_t *tmp,
                                   uint32_t &flags) {
  const uint32_t blen = wide_len(bound, bw);
  for (uint32_t j = 0; j < bw; ++j) r[j] = 0;
  if (blen == 0) {  // unreachable for consistent counts
    flags |= FLAG_CAPACITY;
    return;
  }
  if (blen == 1 && bound[0] == 1) return;
  for (uint32_t j = 0; j < blen; ++j) tmp[j] = bound[j];
  for (uint32_t j = 0; j < blen; ++j) {  // tmp = bound - 1
    if (tmp[j] != 0) {
      tmp[j] -= 1;
      break;
    }
    tmp[j] = ~0ULL;
  }
  const uint32_t tw = wide_len(tmp, blen);
  const uint32_t W = 64 * (tw - 1) + (64 - (uint32_t)__clzll(tmp[tw - 1]));
  const uint32_t q = (W + 63) / 64;
  const uint32_t top = W - 64 * (q - 1);
  const uint64_t mask = top == 64 ? ~0ULL : ((1ULL << top) - 1);
  for (uint32_t a = 0; a < MAX_ATTEMPTS; ++a) {
    uint64_t w[4];
    for (uint32_t j = 0; j < q; ++j) {
      if ((j & 3) == 0) philox4(i, sword, a, j / 4, seed, 0, w);
      r[j] = w[j & 3];
    }
    r[q - 1] &= mask;
    if (wide_cmp(r, bw, bound, bw) < 0) return;
  }
  flags |= FLAG_RNG;
  for (uint32_t j = 0; j < bw; ++j) r[j] = 0;
}

constexpr int WCHUNK = 2 * WB;  // frontier nodes staged per pass

// acc (+)= the sum of the counts of nodes idx[q], q < np (np <= 4), of the level before,
// four limbs at a time in registers so that the loads of a chunk overlap; with first
// the old contents of acc are ignored.  Both levels are limb-major: limb j of acc at
// acc[j * apitch] (j < stride), limb j of node q at src[j * spitch + q] (j < wl).
// wl < stride, so the sum fits.  Returns the width of acc afterwards (its highest nonzero
// limb + 1).
__device__ uint32_t pull_add(uint64_t *__restrict__ acc, uint32_t apitch, uint32_t stride,
                             const uint64_t *__restrict__ src, uint32_t spitch, uint32_t wl,
                             const uint32_t *idx, uint32_t np, bool first) {
  uint32_t width = 0;
  uint64_t carry = 0;  // carry into the next limb (at most np)
  for (uint32_t c0 = 0; c0 < stride; c0 += 4) {
    uint64_t v[4], x[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v[j] = (!first && c0 + j < stride) ? acc[(size_t)(c0 + j) * apitch] : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        x[q][j] = ((uint32_t)q < np && c0 + j < wl) ? src[(size_t)(c0 + j) * spitch + idx[q]] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint64_t sum = v[j] + carry;
      uint64_t c = sum < carry ? 1u : 0u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sum += x[q][j];
        c += sum < x[q][j] ? 1u : 0u;
      }
      v[j] = sum;
      carry = c;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (c0 + j < stride) {
        acc[(size_t)(c0 + j) * apitch] = v[j];
        if (v[j] != 0) width = c0 + j + 1;
      }
  }
  return width;
}

struct WideLds {
  uint32_t k, seg, s, t, flags;
  uint32_t lvl[2];
  uint32_t nvis, pi_count, maxw, maxw_all, sel;
  uint32_t kcount, kfound;
  uint64_t deg[2], new_deg, arcs, top;
  uint64_t skey, kmask, kwant;  // the chosen candidate edge; the radix select's digits so far
  uint32_t c_node[WCHUNK], c_start[WCHUNK], c_pref[WCHUNK + 1];
  uint32_t red[WNW];
};

// Level tables of a wide slot: fields of level l of side x at lv[(x * max_lev + l) * 4 + f].
enum : uint32_t { LV_LO = 0, LV_HI = 1, LV_STRIDE = 2, LV_WIDTH = 3 };

// list == nullptr: every launch index below all_count.
template <bool MULTI>
__global__ __launch_bounds__(WB) void wide_kernel(GraphDev g0, const SampleSeg *__restrict__ segs,
                                                  uint32_t nseg_a, uint64_t seed_a,
                                                  uint32_t phase_a, uint64_t first_a,
                                                  SlotState st, WideState ws,
                                                  const uint32_t *list,
                                                  const uint32_t *list_count, uint32_t all_a,
                                                  uint32_t *work, SampleOut out_a,
                                                  const BatchDesc *__restrict__ bd) {
  __shared__ WideLds L;
  SampleOut out = out_a;
  if (bd && bd->stride) out.stride = bd->stride;
  const uint64_t seed0 = bd ? bd->seed : seed_a, first0 = bd ? bd->first : first_a;
  const uint32_t phase0 = bd ? bd->phase : phase_a, all_count = bd ? bd->count : all_a;
  const uint32_t nseg = bd ? bd->nseg : nseg_a;
  const uint32_t tid = threadIdx.x, wid = tid / WAVE, lane = lane_id();
  const size_t n = st.n;
  const size_t slot = blockIdx.x;
  uint32_t *rec = st.rec + slot * n * REC_WORDS;  // tags and node positions
  uint32_t *visit = st.visit + slot * n;
  uint64_t *gpi = st.pi + slot * st.pi_cap;
  uint64_t *arena = ws.arena + slot * ws.arena_limbs;
  uint32_t *lv = ws.lv + slot * 2 * (size_t)ws.max_lev * 4;
  uint64_t *lb = ws.lbase + slot * 2 * (size_t)ws.max_lev;
  const uint32_t nlist = list ? *list_count : all_count;
  auto LV = [&](uint32_t side, uint32_t l, uint32_t f) -> uint32_t & {
    return lv[((size_t)side * ws.max_lev + l) * 4 + f];
  };
  auto LB = [&](uint32_t side, uint32_t l) -> uint64_t & {
    return lb[(size_t)side * ws.max_lev + l];
  };
  for (;;) {
    if (tid == 0) {
      const uint32_t j = atomicAdd(work, 1u);
      L.k = j < nlist ? (list ? list[j] : j) : 0xFFFFFFFFu;
      if (MULTI && L.k != 0xFFFFFFFFu) {
        uint32_t lo = 0, hi = nseg;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (segs[mid].begin <= L.k) lo = mid; else hi = mid;
        }
        L.seg = lo;
      }
    }
    __syncthreads();
    const uint32_t k = L.k;
    if (k == 0xFFFFFFFFu) break;
    GraphDev g = g0;
    uint64_t seed = seed0, i = first0 + k;
    uint32_t phase = phase0, base = 0;
    if (MULTI) {
      const SampleSeg &S = segs[__builtin_amdgcn_readfirstlane(L.seg)];
      g.n = S.n;
      g.row = S.row;
      g.col = S.col;
      g.rrow = S.rrow;
      g.rcol = S.rcol;
      g.forward = S.forward;
      seed = S.seed;
      phase = S.phase;
      i = S.first + (k - S.begin);
      base = S.id_base;
    }
    if (tid == 0) {
      uint32_t fl = 0;
      const uint32_t s = (uint32_t)uniform_below(u128{g.n, 0}, seed, i, stream_word(phase, P_S, 0), fl).lo;
      const uint32_t tp = (uint32_t)uniform_below(u128{g.n - 1u, 0}, seed, i, stream_word(phase, P_T, 0), fl).lo;
      const uint32_t t = tp + (tp >= s ? 1u : 0u);
      L.s = s;
      L.t = t;
      *tag_of(rec, s) = 1u;
      *tag_of(rec, t) = TAG_T | 1u;
      visit[0] = s;
      visit[1] = t;
      *pos_of(rec, s) = 0;
      *pos_of(rec, t) = 1;
      arena[0] = 1;
      arena[1] = 1;
      for (uint32_t x = 0; x < 2; ++x) {
        LV(x, 0, LV_LO) = x;
        LV(x, 0, LV_HI) = x + 1;
        LV(x, 0, LV_STRIDE) = 1;
        LV(x, 0, LV_WIDTH) = 1;
        LB(x, 0) = x;
      }
      L.top = 2;
      L.lvl[0] = 0;
      L.lvl[1] = 0;
      L.deg[0] = (uint64_t)(g.row[s + 1] - g.row[s]);
      L.deg[1] = (uint64_t)(g.rrow[t + 1] - g.rrow[t]);
      L.arcs = 0;
      L.nvis = 2;
      L.flags = fl;
      L.maxw = 0;
      L.maxw_all = 1;
    }
    __syncthreads();
    bool met = false;
    uint32_t needed = 0;
    // the expansion that met: its side, frontier and the other side's tag (uniform)
    uint32_t m_side = 0, m_fb = 0, m_fe = 0, m_otag = 0;
    for (;;) {
      // ties expand the s side; the forward search expands it always
      const uint32_t me = (g.forward || L.deg[0] <= L.deg[1]) ? 0u : 1u;
      const uint32_t ot = 1u - me;
      const uint32_t l = L.lvl[me], lo_ = L.lvl[ot];
      const uint32_t fb = LV(me, l, LV_LO), fe = LV(me, l, LV_HI);
      const uint32_t other_tag = (ot == 0 ? 0u : TAG_T) | (lo_ + 1);
      const uint32_t cur_tag = (me == 0 ? 0u : TAG_T) | (l + 1);
      const uint32_t next_tag = (me == 0 ? 0u : TAG_T) | (l + 2);
      const uint32_t *rp = me == 0 ? g.row : g.rrow;
      const uint32_t *cl = me == 0 ? g.col : g.rcol;
      const uint32_t *pr = me == 0 ? g.rrow : g.row;  // predecessors of the new level
      const uint32_t *pc = me == 0 ? g.rcol : g.col;
      const uint64_t dme = L.deg[me];
      const uint32_t nb = L.nvis;
      const uint32_t wl = LV(me, l, LV_WIDTH);
      const uint64_t bl = LB(me, l);
      const uint32_t stride = wl + 1;
      const uint64_t nbase = L.top;
      needed = nb;
      if (l + 1 >= ws.max_lev) {  // no room for the next level's table entry
        __syncthreads();
        if (tid == 0) L.flags |= FLAG_CAPACITY;
        break;
      }
      __syncthreads();
      if (tid == 0) {
        L.arcs += dme;
        L.pi_count = 0;
        L.new_deg = 0;
        L.maxw = 0;
      }
      __syncthreads();
      // ---- one pass over the frontier's arcs: the meeting test and the claims of the
      // next level's nodes
      for (uint32_t cb = fb; cb < fe; cb += WCHUNK) {
        const uint32_t m = min((uint32_t)WCHUNK, fe - cb);
        uint32_t d[2] = {0, 0};
        for (int q = 0; q < 2; ++q) {
          const uint32_t j = 2 * tid + q;
          if (j < m) {
            const uint32_t u = visit[cb + j];
            const uint32_t st0 = rp[u];
            d[q] = rp[u + 1] - st0;
            L.c_node[j] = u;
            L.c_start[j] = st0;
          }
        }
        // exclusive scan of the staged degrees
        const uint32_t inc = wave_incl_u32(d[0] + d[1]);
        if (lane == WAVE - 1) L.red[wid] = inc;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int q = 0; q < WNW; ++q) {
          if ((uint32_t)q < wid) before += L.red[q];
          tot += L.red[q];
        }
        const uint32_t ex = before + inc - (d[0] + d[1]);
        if (2 * tid < m) L.c_pref[2 * tid] = ex;
        if (2 * tid + 1 < m) L.c_pref[2 * tid + 1] = ex + d[0];
        if (tid == 0) L.c_pref[m] = tot;
        __syncthreads();
        // UA arcs per thread at a time: their row reads, tag loads and claims go out
        // together rather than one arc's after another's
        constexpr int UA = 4;
        for (uint32_t e0 = tid; e0 < tot; e0 += WB * UA) {
          uint32_t uu[UA], ww[UA], tg[UA], old[UA];
#pragma unroll
          for (int q = 0; q < UA; ++q) {
            const uint32_t e = e0 + (uint32_t)q * WB;
            uu[q] = 0xFFFFFFFFu;  // no arc
            ww[q] = 0;
            if (e < tot) {
              uint32_t lo = 0, hi = m;  // largest j with c_pref[j] <= e
              while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (L.c_pref[mid] <= e) lo = mid; else hi = mid;
              }
              uu[q] = L.c_node[lo];
              ww[q] = cl[L.c_start[lo] + (e - L.c_pref[lo])];
            }
          }
#pragma unroll
          for (int q = 0; q < UA; ++q)
            tg[q] = uu[q] != 0xFFFFFFFFu ? ld_tag(tag_of(rec, ww[q])) : next_tag;  // next_tag: skip
#pragma unroll
          for (int q = 0; q < UA; ++q)
            old[q] = tg[q] == 0 ? cas_tag(tag_of(rec, ww[q]), 0u, next_tag) : 1u;
#pragma unroll
          for (int q = 0; q < UA; ++q) {
            const uint32_t u = uu[q], w = ww[q];
            if (tg[q] == other_tag) {
              const uint32_t idx = atomicAdd(&L.pi_count, 1u);
              const uint64_t key = me == 0 ? (((uint64_t)u << 32) | w) : (((uint64_t)w << 32) | u);
              if (idx < st.pi_cap) gpi[idx] = key;
            } else if (tg[q] == 0 && old[q] == 0u) {  // this arc claimed w
              const uint32_t p = atomicAdd(&L.nvis, 1u);
              visit[p] = w;
              *pos_of(rec, w) = p;
              atomicAdd((unsigned long long *)&L.new_deg, (unsigned long long)(rp[w + 1] - rp[w]));
            }
          }
        }
        __syncthreads();
      }
      if (L.pi_count > 0) {  // the level just discovered is never used: no counts for it
        met = true;
        m_side = me;
        m_fb = fb;
        m_fe = fe;
        m_otag = other_tag;
        break;
      }
      const uint32_t ne = L.nvis;
      if (ne == nb) break;  // the expanded side closed: s and t are disconnected
      // ---- the new level's counts, stored limb-major: limb j of the node at position p
      // at arena[nbase + j * (ne - nb) + (p - nb)].  The thread of p pulls it from the
      // node's predecessors on level l (limb j of its node q at arena[bl + j * (fe - fb)
      // + q]), so consecutive threads write consecutive words and read nearby ones.
      const uint32_t mnew = ne - nb, mcur = fe - fb;
      if (nbase + (uint64_t)mnew * stride > ws.arena_limbs) {
        if (tid == 0) L.flags |= FLAG_CAPACITY;
        break;
      }
      uint32_t used_max = 0;
      for (uint32_t p = nb + tid; p < ne; p += WB) {
        const uint32_t w = visit[p];
        uint64_t *acc = arena + nbase + (p - nb);
        uint32_t idx[4], np = 0, width = 0;
        bool first = true;
        const uint32_t pe = pr[w + 1];
        // the node's in-arcs eight at a time: their tails, then the tails' tags and
        // positions (one load each: no claim changes them during this pass), all in flight
        // together; predecessors on level l are added four at a time
        constexpr int UP = 8;
        for (uint32_t e0 = pr[w]; e0 < pe; e0 += UP) {
          uint32_t uu[UP];
          uint2 tp[UP];
#pragma unroll
          for (int q = 0; q < UP; ++q) uu[q] = e0 + q < pe ? pc[e0 + q] : 0xFFFFFFFFu;
#pragma unroll
          for (int q = 0; q < UP; ++q)
            tp[q] = uu[q] != 0xFFFFFFFFu ? *reinterpret_cast<const uint2 *>(tag_of(rec, uu[q]))
                                         : make_uint2(0u, 0u);
#pragma unroll
          for (int q = 0; q < UP; ++q) {
            if (tp[q].x == cur_tag) idx[np++] = tp[q].y - fb;  // (cur_tag is never 0)
            if (np == 4) {
              width = pull_add(acc, mnew, stride, arena + bl, mcur, wl, idx, np, first);
              first = false;
              np = 0;
            }
          }
        }
        if (np > 0 || first)  // the rest (or, with no predecessor, zeros)
          width = pull_add(acc, mnew, stride, arena + bl, mcur, wl, idx, np, first);
        used_max = max(used_max, width);
      }
      atomicMax(&L.maxw, used_max);
      __syncthreads();
      if (tid == 0) {
        const uint32_t wn = max(L.maxw, 1u);
        LV(me, l + 1, LV_LO) = nb;
        LV(me, l + 1, LV_HI) = ne;
        LV(me, l + 1, LV_STRIDE) = stride;
        LV(me, l + 1, LV_WIDTH) = wn;
        LB(me, l + 1) = nbase;
        L.top = nbase + (uint64_t)(ne - nb) * stride;
        L.deg[me] = L.new_deg;
        L.lvl[me] = l + 1;
        L.maxw_all = max(L.maxw_all, wn);
      }
      __syncthreads();
    }
    __syncthreads();
    const uint32_t ls = L.lvl[0], lt = L.lvl[1];
    uint32_t len = 0;
    uint32_t *path = out.path + (size_t)k * out.stride;
    if (met && L.flags == 0) {
      const uint32_t P = L.pi_count;
      const uint32_t ws_ = LV(0, ls, LV_WIDTH), wt_ = LV(1, lt, LV_WIDTH);
      const uint32_t pw = ws_ + wt_;
      const uint32_t tw = max(pw, L.maxw_all) + 2;  // totals, draws, running sums
      constexpr uint32_t GROUPS = WB / 16;  // block sums are combined in groups of 16
      static_assert(WB == GROUPS * 16, "one block of candidate edges per thread");
      const uint32_t so = LV(0, ls, LV_LO), sp = LV(0, ls, LV_HI) - so;  // limb pitches
      const uint32_t to = LV(1, lt, LV_LO), tp = LV(1, lt, LV_HI) - to;
      const uint64_t sb = LB(0, ls), tb = LB(1, lt);
      // weight of candidate edge (v, w): sigma_s(v) sigma_t(w), pw limbs at dst
      auto weight = [&](uint64_t key, uint64_t *dst) {
        const uint32_t v = (uint32_t)(key >> 32), w = (uint32_t)key;
        wide_mul_s(arena + sb + (*pos_of(rec, v) - so), sp, ws_,
                   arena + tb + (*pos_of(rec, w) - to), tp, wt_, dst);
      };
      const uint64_t prod = L.top;  // the (unused) new level's place: free from here on
      uint64_t *bscr = nullptr;     // six numbers of tw limbs for the two backtracking walks
      if (ls + lt + 2 > out.stride) {
        if (tid == 0) L.flags |= FLAG_CAPACITY;
      } else if (P <= st.pi_cap) {
        const uint64_t need = prod + (uint64_t)P * pw + (uint64_t)(WB + GROUPS + 11) * tw;
        if (need > ws.arena_limbs) {
          if (tid == 0) L.flags |= FLAG_CAPACITY;
        } else {
          // ---- candidate edges in canonical order, and their weights
          uint32_t M = 1;
          while (M < P) M <<= 1;
          for (uint32_t j = P + tid; j < M; j += WB) gpi[j] = ~0ULL;
          __syncthreads();
          bitonic_sort<WB>(gpi, M);
          for (uint32_t j = tid; j < P; j += WB) weight(gpi[j], arena + prod + (size_t)j * pw);
          __syncthreads();
          // sums of contiguous blocks of weights (one block per thread), then of groups
          // of 16 blocks, so that the total and the prefix that passes r need few serial adds
          uint64_t *bsum = arena + prod + (size_t)P * pw;
          uint64_t *gsum = bsum + (size_t)WB * tw;
          uint64_t *scr = gsum + (size_t)GROUPS * tw;  // 11 scratch numbers
          bscr = scr + 5 * (size_t)tw;
          const uint32_t b0 = (uint32_t)((uint64_t)P * tid / WB), b1 = (uint32_t)((uint64_t)P * (tid + 1) / WB);
          {
            uint64_t *bs = bsum + (size_t)tid * tw;
            for (uint32_t j = 0; j < tw; ++j) bs[j] = 0;
            for (uint32_t j = b0; j < b1; ++j) (void)wide_add(bs, tw, arena + prod + (size_t)j * pw, pw);
          }
          __syncthreads();
          if (tid < GROUPS) {
            uint64_t *gs = gsum + (size_t)tid * tw;
            for (uint32_t j = 0; j < tw; ++j) gs[j] = 0;
            for (uint32_t b = tid * 16; b < tid * 16 + 16; ++b) (void)wide_add(gs, tw, bsum + (size_t)b * tw, tw);
          }
          __syncthreads();
          if (tid == 0) {
            uint64_t *total = scr, *r = scr + tw, *tmp = scr + 2 * tw, *acc = scr + 3 * tw,
                     *sv = scr + 4 * tw;
            uint32_t fl = 0;
            for (uint32_t j = 0; j < tw; ++j) total[j] = 0;
            for (uint32_t gi = 0; gi < GROUPS; ++gi) (void)wide_add(total, tw, gsum + (size_t)gi * tw, tw);
            uniform_below_wide(total, tw, seed, i, stream_word(phase, P_EDGE, 0), r, tmp, fl);
            // the first edge whose prefix sum passes r: group, then block, then edge
            for (uint32_t j = 0; j < tw; ++j) acc[j] = 0;
            auto step = [&](const uint64_t *x, uint32_t xw) -> bool {  // acc += x unless that passes r
              for (uint32_t j = 0; j < tw; ++j) sv[j] = acc[j];
              (void)wide_add(acc, tw, x, xw);
              if (wide_cmp(acc, tw, r, tw) > 0) {
                for (uint32_t j = 0; j < tw; ++j) acc[j] = sv[j];
                return true;
              }
              return false;
            };
            uint32_t gsel = GROUPS, bsel = WB, sel = P;
            for (uint32_t gi = 0; gi < GROUPS && fl == 0; ++gi)
              if (step(gsum + (size_t)gi * tw, tw)) {
                gsel = gi;
                break;
              }
            for (uint32_t b = gsel * 16; gsel < GROUPS && b < gsel * 16 + 16; ++b)
              if (step(bsum + (size_t)b * tw, tw)) {
                bsel = b;
                break;
              }
            if (bsel < WB) {
              const uint32_t e0 = (uint32_t)((uint64_t)P * bsel / WB), e1 = (uint32_t)((uint64_t)P * (bsel + 1) / WB);
              for (uint32_t j = e0; j < e1; ++j)
                if (step(arena + prod + (size_t)j * pw, pw)) {
                  sel = j;
                  break;
                }
            }
            if (sel >= P) fl |= FLAG_CAPACITY;  // unreachable for consistent counts
            else L.skey = gpi[sel];
            L.flags |= fl;
          }
        }
      } else {
        // ---- more candidate edges than the slot's buffer holds.  Every one is written
        // to the arena by a second pass over the meeting level (its tags are unchanged,
        // so it finds the same edges), and the edge is chosen without sorting: a weighted
        // radix select over the 64-bit keys (v << 32 | w), four bits at a time from the
        // top.  Pass d sums the weights of the keys that agree with the digits chosen so
        // far into 16 buckets by their next digit; the digit taken is the first whose
        // bucket makes the running sum pass r.  The key found is the first key, in
        // ascending order, whose prefix sum of weights passes r -- the canonical choice.
        constexpr uint32_t NB = 16;
        uint64_t *keys = arena + prod;
        uint64_t *part = keys + P;                     // WB x NB numbers: per-thread buckets
        uint64_t *l2 = part + (size_t)WB * NB * tw;    // WB numbers: partial bucket sums
        uint64_t *bsum = l2 + (size_t)WB * tw;         // NB numbers: bucket sums
        uint64_t *scr = bsum + (size_t)NB * tw;        // total, r, tmp, below, saved; 6 more
        uint64_t *prodt = scr + 11 * (size_t)tw;       // WB products of pw limbs
        bscr = scr + 5 * (size_t)tw;
        const uint64_t need = (uint64_t)(prodt - arena) + (uint64_t)WB * pw;
        if (need > ws.arena_limbs) {
          if (tid == 0) L.flags |= FLAG_CAPACITY;
        } else {
          const uint32_t *rp = m_side == 0 ? g.row : g.rrow;
          const uint32_t *cl = m_side == 0 ? g.col : g.rcol;
          if (tid == 0) {
            L.kcount = 0;
            L.kmask = 0;
            L.kwant = 0;
          }
          __syncthreads();
          for (uint32_t cb = m_fb; cb < m_fe; cb += WCHUNK) {
            const uint32_t m = min((uint32_t)WCHUNK, m_fe - cb);
            uint32_t d[2] = {0, 0};
            for (int q = 0; q < 2; ++q) {
              const uint32_t j = 2 * tid + q;
              if (j < m) {
                const uint32_t u = visit[cb + j];
                const uint32_t st0 = rp[u];
                d[q] = rp[u + 1] - st0;
                L.c_node[j] = u;
                L.c_start[j] = st0;
              }
            }
            const uint32_t inc = wave_incl_u32(d[0] + d[1]);
            if (lane == WAVE - 1) L.red[wid] = inc;
            __syncthreads();
            uint32_t before = 0, tot = 0;
            for (int q = 0; q < WNW; ++q) {
              if ((uint32_t)q < wid) before += L.red[q];
              tot += L.red[q];
            }
            const uint32_t ex = before + inc - (d[0] + d[1]);
            if (2 * tid < m) L.c_pref[2 * tid] = ex;
            if (2 * tid + 1 < m) L.c_pref[2 * tid + 1] = ex + d[0];
            if (tid == 0) L.c_pref[m] = tot;
            __syncthreads();
            for (uint32_t e = tid; e < tot; e += WB) {
              uint32_t lo = 0, hi = m;  // largest j with c_pref[j] <= e
              while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (L.c_pref[mid] <= e) lo = mid; else hi = mid;
              }
              const uint32_t u = L.c_node[lo];
              const uint32_t w = cl[L.c_start[lo] + (e - L.c_pref[lo])];
              if (ld_tag(tag_of(rec, w)) == m_otag) {
                const uint32_t idx = atomicAdd(&L.kcount, 1u);
                const uint64_t key = m_side == 0 ? (((uint64_t)u << 32) | w) : (((uint64_t)w << 32) | u);
                if (idx < P) keys[idx] = key;
              }
            }
            __syncthreads();
          }
          if (L.kcount != P) {  // unreachable: the same level, the same tags
            if (tid == 0) L.flags |= FLAG_CAPACITY;
          } else {
            uint32_t nbits = 1;  // both halves of a key are below n: bits [0, 4D) each
            while (nbits < 32 && ((g.n - 1u) >> nbits) != 0) ++nbits;
            const uint32_t D = (nbits + 3) / 4;
            uint64_t *mypart = part + (size_t)tid * NB * tw;
            uint64_t *myprod = prodt + (size_t)tid * pw;
            for (uint32_t pass = 0; pass < 2 * D; ++pass) {
              const uint32_t sh = (pass < D ? 32u : 0u) + 4u * (D - 1u - pass % D);
              const uint64_t kmask = L.kmask, kwant = L.kwant;
              for (uint32_t j = 0; j < NB * tw; ++j) mypart[j] = 0;
              for (uint32_t j = tid; j < P; j += WB) {
                const uint64_t key = keys[j];
                if ((key & kmask) != kwant) continue;
                weight(key, myprod);
                (void)wide_add(mypart + (size_t)((key >> sh) & (NB - 1)) * tw, tw, myprod, pw);
              }
              __syncthreads();
              {  // bucket tid % NB over threads [16 (tid / NB), +16)
                const uint32_t b = tid % NB, t0 = (tid / NB) * 16;
                uint64_t *acc = l2 + (size_t)tid * tw;
                for (uint32_t j = 0; j < tw; ++j) acc[j] = 0;
                for (uint32_t t = t0; t < t0 + 16; ++t)
                  (void)wide_add(acc, tw, part + ((size_t)t * NB + b) * tw, tw);
              }
              __syncthreads();
              if (tid < NB) {  // bucket tid: the WB / NB partial sums of the threads above
                uint64_t *acc = bsum + (size_t)tid * tw;
                for (uint32_t j = 0; j < tw; ++j) acc[j] = 0;
                for (uint32_t q = tid; q < (uint32_t)WB; q += NB)
                  (void)wide_add(acc, tw, l2 + (size_t)q * tw, tw);
              }
              __syncthreads();
              if (tid == 0) {
                uint64_t *total = scr, *r = scr + tw, *tmp = scr + 2 * tw, *below = scr + 3 * tw,
                         *sv = scr + 4 * tw;
                uint32_t fl = 0;
                if (pass == 0) {
                  for (uint32_t j = 0; j < tw; ++j) total[j] = 0;
                  for (uint32_t b = 0; b < NB; ++b) (void)wide_add(total, tw, bsum + (size_t)b * tw, tw);
                  uniform_below_wide(total, tw, seed, i, stream_word(phase, P_EDGE, 0), r, tmp, fl);
                  for (uint32_t j = 0; j < tw; ++j) below[j] = 0;
                }
                uint32_t pick = NB;
                for (uint32_t b = 0; b < NB && fl == 0; ++b) {
                  for (uint32_t j = 0; j < tw; ++j) sv[j] = below[j];
                  (void)wide_add(below, tw, bsum + (size_t)b * tw, tw);
                  if (wide_cmp(below, tw, r, tw) > 0) {
                    for (uint32_t j = 0; j < tw; ++j) below[j] = sv[j];
                    pick = b;
                    break;
                  }
                }
                if (pick == NB) fl |= FLAG_CAPACITY;  // unreachable: r < total
                L.kmask = kmask | ((uint64_t)(NB - 1) << sh);
                L.kwant = kwant | ((uint64_t)(pick & (NB - 1)) << sh);
                L.flags |= fl;
              }
              __syncthreads();
              if (L.flags) break;
            }
            if (L.flags == 0) {  // the digits name one key of the list (keys are distinct)
              if (tid == 0) L.kfound = 0;
              __syncthreads();
              const uint64_t kw = L.kwant;
              for (uint32_t j = tid; j < P; j += WB)
                if (keys[j] == kw) atomicAdd(&L.kfound, 1u);
              __syncthreads();
              if (tid == 0) {
                if (L.kfound == 1) L.skey = kw;
                else L.flags |= FLAG_CAPACITY;  // unreachable
              }
            }
          }
        }
      }
      __syncthreads();
      // ---- backtracking (section 4): the two sides at once, by lane 0 of waves 0 and 1
      if (L.flags == 0 && (tid == 0 || tid == WAVE)) {
        const uint32_t side = tid == 0 ? 0u : 1u;
        uint64_t *r = bscr + (size_t)(3 * side) * tw;
        uint64_t *acc = r + tw, *tmp2 = r + 2 * tw;
        uint32_t fl = 0;
        const uint64_t key = L.skey;
        uint32_t x = side == 0 ? (uint32_t)(key >> 32) : (uint32_t)key;
        const uint32_t lev = side == 0 ? ls : lt;
        path[side == 0 ? ls : ls + 1] = x + base;
        const uint32_t *brp = side == 0 ? g.rrow : g.row;
        const uint32_t *bcl = side == 0 ? g.rcol : g.col;
        for (uint32_t j = lev; j >= 1 && fl == 0; --j) {
          const uint32_t xw = LV(side, j, LV_WIDTH), xlo = LV(side, j, LV_LO);
          const uint64_t *sx = arena + LB(side, j) + (*pos_of(rec, x) - xlo);
          const uint32_t xp = LV(side, j, LV_HI) - xlo;  // limb pitch of level j
          for (uint32_t q = 0; q < xw; ++q) acc[q] = sx[(size_t)q * xp];  // sigma(x)
          uniform_below_wide(acc, xw, seed, i,
                             stream_word(phase, side == 0 ? P_BACK_S : P_BACK_T, j), r, tmp2, fl);
          const uint32_t want = (side == 0 ? 0u : TAG_T) | j;  // level j-1
          const uint32_t pwid = LV(side, j - 1, LV_WIDTH), plo = LV(side, j - 1, LV_LO);
          const uint32_t ppt = LV(side, j - 1, LV_HI) - plo;  // limb pitch of level j-1
          const uint64_t pb = LB(side, j - 1);
          for (uint32_t q = 0; q < tw; ++q) acc[q] = 0;
          uint32_t pick = 0xFFFFFFFFu;
          for (uint32_t e = brp[x]; e < brp[x + 1] && fl == 0; ++e) {
            const uint32_t u = bcl[e];
            if (ld_tag(tag_of(rec, u)) != want) continue;
            wide_add_s(acc, tw, arena + pb + (*pos_of(rec, u) - plo), ppt, pwid);
            if (wide_cmp(acc, tw, r, xw) > 0) {
              pick = u;
              break;
            }
          }
          if (pick == 0xFFFFFFFFu) {
            fl |= FLAG_CAPACITY;  // unreachable for consistent counts
            break;
          }
          x = pick;
          path[side == 0 ? j - 1 : ls + 1 + (lev - j) + 1] = x + base;
        }
        if (fl) atomicOr(&L.flags, fl);
      }
      __syncthreads();
      if (L.flags == 0) len = ls + lt + 2;
    }
    __syncthreads();
    if (tid == 0) {
      out.s[k] = L.s;
      out.t[k] = L.t;
      out.len[k] = L.flags ? 0u : len;
      out.arcs[k] = L.arcs;
      out.flags[k] = L.flags;
      out.nodes[k] = needed;
      // a sample that outgrew this launch's arena is sampled again by a launch with
      // larger arenas (when the caller keeps a list)
      if ((L.flags & FLAG_CAPACITY) && out.fix_list)
        out.fix_list[atomicAdd(out.fix_count, 1u)] = k;
    }
    // ---- restore the slot's all-zero state
    const uint32_t nv = L.nvis;
    for (uint32_t j = tid; j < nv; j += WB) {
      const uint32_t v = visit[j];
      *tag_of(rec, v) = 0;
      *pos_of(rec, v) = 0;
    }
    __syncthreads();
  }
}

// *arcs_total += the sum of arcs[0, count); *flags_or |= the OR of flags[0, count).
__global__ __launch_bounds__(256) void sample_sums_kernel(const uint64_t *__restrict__ arcs,
                                                          const uint32_t *__restrict__ flags,
                                                          uint32_t count, uint64_t *arcs_total,
                                                          uint32_t *flags_or) {
  __shared__ uint64_t sa[256 / WAVE];
  __shared__ uint32_t sf[256 / WAVE];
  uint64_t a = 0;
  uint32_t f = 0;
  for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < count; k += gridDim.x * 256) {
    a += arcs[k];
    f |= flags[k];
  }
  a = wave_sum_u64(a);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) f |= __shfl_xor(f, d, WAVE);
  if (lane_id() == 0) {
    sa[threadIdx.x / WAVE] = a;
    sf[threadIdx.x / WAVE] = f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / WAVE; ++w) {
      a += sa[w];
      f |= sf[w];
    }
    if (a) atomicAdd((unsigned long long *)arcs_total, (unsigned long long)a);
    if (f) atomicOr(flags_or, f);
  }
}

// The fixed working memory of the calls that allocate nothing (see noalloc_scratch).
static __device__ __align__(256) uint64_t scratch[NOALLOC_SCRATCH_BYTES / 8];

}  // namespace

template <bool MULTI, bool HASHED>
hipError_t launch_sampler_shape(int block, uint32_t grid, hipStream_t stream, const GraphDev &g,
                                const SlotState &st, uint64_t seed, uint32_t phase,
                                uint64_t first, const SampleSeg *segs, uint32_t nseg,
                                uint32_t count, uint32_t *work, const SampleOut &out,
                                uint32_t small_exp, const BatchDesc *bd) {
  switch (block) {
    case 64:
      hipLaunchKernelGGL((sampler_kernel<64, MULTI, HASHED>), dim3(grid), dim3(64), 0, stream, g,
                         st, seed, phase, first, segs, nseg, count, work, out, small_exp, bd);
      break;
    case 128:
      hipLaunchKernelGGL((sampler_kernel<128, MULTI, HASHED>), dim3(grid), dim3(128), 0, stream,
                         g, st, seed, phase, first, segs, nseg, count, work, out, small_exp, bd);
      break;
    case 256:
      hipLaunchKernelGGL((sampler_kernel<256, MULTI, HASHED>), dim3(grid), dim3(256), 0, stream,
                         g, st, seed, phase, first, segs, nseg, count, work, out, small_exp, bd);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Slot tables (st.hbits in [1, 31]: hashed records) or one record per node (0).
template <bool MULTI>
hipError_t launch_sampler_variant(int block, uint32_t grid, hipStream_t stream, const GraphDev &g,
                                  const SlotState &st, uint64_t seed, uint32_t phase,
                                  uint64_t first, const SampleSeg *segs, uint32_t nseg,
                                  uint32_t count, uint32_t *work, const SampleOut &out,
                                  uint32_t small_exp, const BatchDesc *bd) {
  if (st.hbits > 31 || (st.hbits != 0 && (!st.vh || st.n != (1u << st.hbits))))
    return hipErrorInvalidValue;
  if (st.hbits)
    return launch_sampler_shape<MULTI, true>(block, grid, stream, g, st, seed, phase, first,
                                             segs, nseg, count, work, out, small_exp, bd);
  return launch_sampler_shape<MULTI, false>(block, grid, stream, g, st, seed, phase, first, segs,
                                            nseg, count, work, out, small_exp, bd);
}

hipError_t launch_sampler(const GraphDev &g, const SlotState &st, uint64_t seed, uint32_t phase,
                          uint64_t first, uint32_t count, uint32_t *work, const SampleOut &out,
                          uint32_t grid, const LaunchShape &shape, hipStream_t stream,
                          const BatchDesc *bd) {
  if (count == 0) return hipSuccess;
  if ((st.hbits == 0 && st.n < g.n) || grid > st.slots || grid == 0) return hipErrorInvalidValue;
  return launch_sampler_variant<false>(shape.block, grid, stream, g, st, seed, phase, first,
                                       nullptr, 0u, count, work, out, shape.small_exp, bd);
}

hipError_t launch_sampler_multi(const SampleSeg *segs, uint32_t nseg, const SlotState &st,
                                uint32_t count, uint32_t *work, const SampleOut &out,
                                uint32_t grid, const LaunchShape &shape, hipStream_t stream,
                                const BatchDesc *bd) {
  if (count == 0) return hipSuccess;
  if (nseg == 0 || grid > st.slots || grid == 0) return hipErrorInvalidValue;
  GraphDev none{};
  return launch_sampler_variant<true>(shape.block, grid, stream, none, st, 0ull, 0u, 0ull, segs,
                                      nseg, count, work, out, shape.small_exp, bd);
}

hipError_t launch_wide_fix(const GraphDev &g, uint64_t seed, uint32_t phase, uint64_t first,
                           const SampleSeg *segs, uint32_t nseg, const SlotState &st,
                           const WideState &ws, uint32_t count, bool all,
                           const uint32_t *list, const uint32_t *list_count, uint32_t *work,
                           const SampleOut &out, hipStream_t stream, const BatchDesc *bd) {
  if (count == 0) return hipSuccess;
  if (ws.slots == 0 || ws.slots > st.slots || !ws.arena || !work) return hipErrorInvalidValue;
  if (!all && (!list || !list_count)) return hipErrorInvalidValue;
  const uint32_t *lst = all ? nullptr : list;
  if (segs)
    hipLaunchKernelGGL(wide_kernel<true>, dim3(ws.slots), dim3(WB), 0, stream, g, segs, nseg,
                       seed, phase, first, st, ws, lst, list_count, count, work, out, bd);
  else
    hipLaunchKernelGGL(wide_kernel<false>, dim3(ws.slots), dim3(WB), 0, stream, g, segs, nseg,
                       seed, phase, first, st, ws, lst, list_count, count, work, out, bd);
  return hipGetLastError();
}

// The same reduction for the hits of one check interval: count[v] += 1 per interior hit
// by a device atomic, and the group maximum is raised to the count the atomic returned
// plus one -- the largest of those for a node is its final count, so counts and maxima
// equal the tiled reduction's.  One kernel and no LDS: a run reduces a batch's check
// intervals one after another, and this chain is on its critical path.
__global__ __launch_bounds__(HIT_BLOCK) void hit_atomic_kernel(const uint32_t *path,
                                                               const uint32_t *len,
                                                               uint32_t stride, uint32_t nsamp,
                                                               uint32_t n, uint64_t *count,
                                                               const uint32_t *group,
                                                               uint64_t *gmax) {
  const uint64_t entries = (uint64_t)nsamp * stride;
  for (uint64_t e = (uint64_t)blockIdx.x * HIT_BLOCK + threadIdx.x; e < entries;
       e += (uint64_t)gridDim.x * HIT_BLOCK) {
    const uint32_t k = (uint32_t)(e / stride), j = (uint32_t)(e % stride);
    if (j < 1 || j + 1 >= len[k]) continue;
    const uint32_t v = path[e];
    if (v >= n) continue;
    const uint64_t c = (uint64_t)atomicAdd((unsigned long long *)&count[v], 1ull) + 1u;
    if (gmax) {
      unsigned long long *gm = (unsigned long long *)&gmax[group[v]];
      if (c > __hip_atomic_load(gm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(gm, (unsigned long long)c);
    }
  }
}

// Additions of at most this many interior hits take the atomic kernel; subtractions and
// larger calls (where hot nodes would serialise many atomics) the tiled kernels.
constexpr uint64_t ATOMIC_MAX_HITS = 1u << 17;

hipError_t launch_hit_reduce(const uint32_t *path, const uint32_t *len, uint32_t stride,
                             uint32_t nsamp, uint32_t n, uint64_t *count, bool subtract,
                             const uint32_t *group, uint64_t *gmax, const HitScratch &hs,
                             hipStream_t stream) {
  if (nsamp == 0) return hipSuccess;
  if (!subtract && (uint64_t)nsamp * (stride > 2 ? stride - 2 : 1) <= ATOMIC_MAX_HITS) {
    const uint64_t entries = (uint64_t)nsamp * stride;
    const uint32_t blocks =
        (uint32_t)std::min<uint64_t>((entries + HIT_BLOCK - 1) / HIT_BLOCK, 1024);
    hipLaunchKernelGGL(hit_atomic_kernel, dim3(blocks), dim3(HIT_BLOCK), 0, stream, path, len,
                       stride, nsamp, n, count, group, gmax);
    return hipGetLastError();
  }
  const uint32_t tiles = (n + HIT_TILE - 1) / HIT_TILE;
  const uint32_t inner = stride > 2 ? stride - 2 : 1;  // most interior nodes of a path
  if (tiles > MAX_HIT_TILES || (uint64_t)nsamp * inner > hs.cap) return hipErrorInvalidValue;
  const bool compact = hs.tile_start != nullptr;
  if (compact && (!hs.tile_fill || hs.cap > 0xFFFFFFFFull)) return hipErrorInvalidValue;
  const bool aggregate = inner <= AGG_SLOTS / 2;
  const uint32_t spp = aggregate ? max(1u, min(SAMPLES_PER_PART, (AGG_SLOTS / 2) / inner)) : 1u;
  const dim3 pgrid((nsamp + spp - 1) / spp);
  if (!compact) {
    hipLaunchKernelGGL(hit_partition_kernel, pgrid, dim3(HIT_BLOCK), 0, stream, path, len, stride,
                       nsamp, tiles, spp, aggregate ? 1 : 0, (int)PASS_FIXED, hs.bins, hs.cap,
                       hs.bin_count, (const uint32_t *)nullptr, (uint32_t *)nullptr);
  } else {
    hipLaunchKernelGGL(hit_partition_kernel, pgrid, dim3(HIT_BLOCK), 0, stream, path, len, stride,
                       nsamp, tiles, spp, aggregate ? 1 : 0, (int)PASS_COUNT, hs.bins, hs.cap,
                       hs.bin_count, (const uint32_t *)hs.tile_start, hs.tile_fill);
    hipLaunchKernelGGL(hit_scan_kernel, dim3(1), dim3(HIT_BLOCK), 0, stream,
                       (const uint32_t *)hs.bin_count, tiles, hs.tile_start);
    hipLaunchKernelGGL(hit_partition_kernel, pgrid, dim3(HIT_BLOCK), 0, stream, path, len, stride,
                       nsamp, tiles, spp, aggregate ? 1 : 0, (int)PASS_WRITE, hs.bins, hs.cap,
                       hs.bin_count, (const uint32_t *)hs.tile_start, hs.tile_fill);
  }
  hipLaunchKernelGGL(hit_tile_kernel, dim3(tiles), dim3(HIT_BLOCK), 0, stream, hs.bins, hs.cap,
                     hs.bin_count, (const uint32_t *)hs.tile_start, hs.tile_fill, n, count,
                     subtract ? 1 : 0, group, gmax);
  return hipGetLastError();
}

// Every check interval of a batch at once (launch_hit_batch).  iv_count_kernel counts
// each node's interior hits per interval in tmp[interval * n + node]; iv_prefix_kernel
// walks each node's intervals in order, adds its hits to its count and raises the
// interval's group maximum to the count the node reached there (clearing tmp);
// iv_snap_kernel takes, per group, the running maximum over the intervals starting from
// the maximum before the batch -- a group's largest count after interval c is that of a
// node hit by then (its count at its last hit) or the earlier maximum -- and writes one
// snapshot per interval (clearing the per-interval maxima).
__global__ __launch_bounds__(HIT_BLOCK) void iv_count_kernel(const uint32_t *path,
                                                             const uint32_t *len,
                                                             uint32_t stride, uint32_t nsamp_a,
                                                             uint32_t per_iv, uint32_t n,
                                                             uint32_t *tmp,
                                                             const BatchDesc *__restrict__ bd) {
  const uint32_t nsamp = bd ? bd->count : nsamp_a;
  const uint64_t entries = (uint64_t)nsamp * stride;
  for (uint64_t e = (uint64_t)blockIdx.x * HIT_BLOCK + threadIdx.x; e < entries;
       e += (uint64_t)gridDim.x * HIT_BLOCK) {
    const uint32_t k = (uint32_t)(e / stride), j = (uint32_t)(e % stride);
    if (j < 1 || j + 1 >= len[k]) continue;
    const uint32_t v = path[e];
    if (v < n) atomicAdd(&tmp[(size_t)(k / per_iv) * n + v], 1u);
  }
}

__global__ __launch_bounds__(HIT_BLOCK) void iv_prefix_kernel(uint32_t n, uint32_t niv_a,
                                                              uint32_t *tmp, uint64_t *count,
                                                              const uint32_t *group,
                                                              uint32_t ngroups,
                                                              uint64_t *ivmax,
                                                              const BatchDesc *__restrict__ bd) {
  const uint32_t niv = bd ? bd->niv : niv_a;
  for (uint32_t v = blockIdx.x * HIT_BLOCK + threadIdx.x; v < n; v += gridDim.x * HIT_BLOCK) {
    uint64_t c = 0;
    bool hit = false;
    for (uint32_t q = 0; q < niv; ++q) {
      const uint32_t h = tmp[(size_t)q * n + v];
      if (h == 0) continue;
      if (!hit) c = count[v];
      hit = true;
      tmp[(size_t)q * n + v] = 0;
      c += h;
      unsigned long long *m = (unsigned long long *)&ivmax[(size_t)q * ngroups + group[v]];
      if (c > __hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(m, (unsigned long long)c);
    }
    if (hit) count[v] = c;
  }
}

__global__ __launch_bounds__(HIT_BLOCK) void iv_snap_kernel(uint32_t niv_a, uint32_t ngroups,
                                                            uint64_t *ivmax, uint64_t *gmax,
                                                            uint64_t *snap,
                                                            const BatchDesc *__restrict__ bd) {
  const uint32_t niv = bd ? bd->niv : niv_a;
  for (uint32_t g = blockIdx.x * HIT_BLOCK + threadIdx.x; g < ngroups;
       g += gridDim.x * HIT_BLOCK) {
    uint64_t m = gmax[g];
    for (uint32_t q = 0; q < niv; ++q) {
      const size_t i = (size_t)q * ngroups + g;
      m = max(m, ivmax[i]);
      ivmax[i] = 0;
      snap[i] = m;
    }
    gmax[g] = m;
  }
}

hipError_t launch_hit_batch(const uint32_t *path, const uint32_t *len, uint32_t stride,
                            uint32_t nsamp, uint32_t per_iv, uint32_t n, uint64_t *count,
                            const uint32_t *group, uint64_t *gmax, uint32_t ngroups,
                            uint32_t *tmp, uint64_t *ivmax, uint64_t *snap,
                            hipStream_t stream, const BatchDesc *bd) {
  if (nsamp == 0) return hipSuccess;
  if (per_iv == 0 || !group || !gmax || !tmp || !ivmax || !snap) return hipErrorInvalidValue;
  const uint32_t niv = (nsamp + per_iv - 1) / per_iv;
  const uint64_t entries = (uint64_t)nsamp * stride;
  const uint32_t b1 = (uint32_t)std::min<uint64_t>((entries + HIT_BLOCK - 1) / HIT_BLOCK, 4096);
  hipLaunchKernelGGL(iv_count_kernel, dim3(b1), dim3(HIT_BLOCK), 0, stream, path, len, stride,
                     nsamp, per_iv, n, tmp, bd);
  const uint32_t b2 = std::min<uint32_t>((n + HIT_BLOCK - 1) / HIT_BLOCK, 4096);
  hipLaunchKernelGGL(iv_prefix_kernel, dim3(b2), dim3(HIT_BLOCK), 0, stream, n, niv, tmp, count,
                     group, ngroups, ivmax, bd);
  const uint32_t b3 = std::max<uint32_t>(1, std::min<uint32_t>((ngroups + HIT_BLOCK - 1) / HIT_BLOCK, 1024));
  hipLaunchKernelGGL(iv_snap_kernel, dim3(b3), dim3(HIT_BLOCK), 0, stream, niv, ngroups, ivmax,
                     gmax, snap, bd);
  return hipGetLastError();
}

hipError_t launch_hit_add_atomic(const uint32_t *path, const uint32_t *len, uint32_t stride,
                                 uint32_t nsamp, uint32_t n, uint64_t *count,
                                 hipStream_t stream) {
  if (nsamp == 0) return hipSuccess;
  const uint64_t entries = (uint64_t)nsamp * stride;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((entries + HIT_BLOCK - 1) / HIT_BLOCK, 1024);
  hipLaunchKernelGGL(hit_atomic_kernel, dim3(blocks), dim3(HIT_BLOCK), 0, stream, path, len,
                     stride, nsamp, n, count, (const uint32_t *)nullptr, (uint64_t *)nullptr);
  return hipGetLastError();
}

hipError_t launch_sample_sums(const uint64_t *arcs, const uint32_t *flags, uint32_t count,
                              uint64_t *arcs_total, uint32_t *flags_or, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const uint32_t blocks = std::min<uint32_t>((count + 255) / 256, 256);
  hipLaunchKernelGGL(sample_sums_kernel, dim3(blocks), dim3(256), 0, stream, arcs, flags, count,
                     arcs_total, flags_or);
  return hipGetLastError();
}

// The device address of `scratch` on the current device, looked up once per device (each
// device holds its own copy of the array, at its own address; in host code the array's
// name is only a stand-in and must never be passed to a kernel).
hipError_t noalloc_scratch(void **ptr) {
  static std::mutex mu;
  static void *addr[NOALLOC_MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// Edge betweenness: every path rewritten as the ids of its edges, with one placeholder
// entry before and after, so that the hit reductions -- which skip a path's first and last
// entry -- count exactly the path's edges.  Step j of sample k (nodes a = path[j], b =
// path[j + 1]) becomes epath[k * estride + 1 + j] = the id of the arc a -> b: its CSR
// position (binary search in a's sorted row), mapped through eid when given (undirected
// graphs: both arcs of an edge share one id).  elen[k] = len[k] + 1, or 0 without a path.
__global__ __launch_bounds__(256) void edge_path_kernel(const uint32_t *__restrict__ path,
                                                        const uint32_t *__restrict__ len,
                                                        uint32_t stride, uint32_t nsamp,
                                                        const uint32_t *__restrict__ row,
                                                        const uint32_t *__restrict__ col,
                                                        const uint32_t *__restrict__ eid,
                                                        uint32_t *epath, uint32_t *elen,
                                                        uint32_t estride,
                                                        const BatchDesc *__restrict__ bd) {
  const uint32_t steps = stride - 1;
  if (bd) nsamp = bd->count;
  const uint64_t total = (uint64_t)nsamp * steps;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * 256) {
    const uint32_t k = (uint32_t)(e / steps), j = (uint32_t)(e % steps);
    const uint32_t L = len[k];
    uint32_t *ep = epath + (size_t)k * estride;
    if (j == 0) {
      elen[k] = L >= 2 ? L + 1 : 0u;
      if (L >= 2) {
        ep[0] = 0;
        ep[L] = 0;
      }
    }
    if (j + 1 < L) {
      const uint32_t a = path[(size_t)k * stride + j], b = path[(size_t)k * stride + j + 1];
      uint32_t lo = row[a], hi = row[a + 1];
      while (lo < hi) {  // first position whose head is not below b (b is in the row)
        const uint32_t mid = (lo + hi) >> 1;
        if (col[mid] < b) lo = mid + 1; else hi = mid;
      }
      ep[1 + j] = eid ? eid[lo] : lo;
    }
  }
}

hipError_t launch_edge_paths(const uint32_t *path, const uint32_t *len, uint32_t stride,
                             uint32_t nsamp, const uint32_t *row, const uint32_t *col,
                             const uint32_t *eid, uint32_t *epath, uint32_t *elen,
                             uint32_t estride, hipStream_t stream, const BatchDesc *bd) {
  if (nsamp == 0) return hipSuccess;
  if (stride < 2 || estride < stride + 1) return hipErrorInvalidValue;
  const uint64_t total = (uint64_t)nsamp * (stride - 1);
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(edge_path_kernel, dim3(blocks), dim3(256), 0, stream, path, len, stride,
                     nsamp, row, col, eid, epath, elen, estride, bd);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, p, count, value);
  return hipGetLastError();
}

hipError_t launch_count_hist(const uint64_t *count, uint32_t n, uint32_t *hist, uint32_t bins,
                             hipStream_t stream) {
  if (n == 0 || bins == 0) return hipSuccess;
  const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(count_hist_kernel, dim3(blocks), dim3(256), 0, stream, count, n, hist, bins);
  return hipGetLastError();
}

hipError_t launch_group_map(const uint64_t *count, uint32_t n, const uint32_t *cgrp, uint32_t bins,
                            uint32_t *group, hipStream_t stream) {
  if (n == 0 || bins == 0) return hipSuccess;
  const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(group_map_kernel, dim3(blocks), dim3(256), 0, stream, count, n, cgrp, bins,
                     group);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint64_t count, hipStream_t stream) {
  return launch_fill_u32(p, count, 0u, stream);
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, uint64_t count,
                              hipStream_t stream, const BatchDesc *bd, uint32_t per,
                              bool by_nseg) {
  if (count == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(copy_kernel<uint32_t>, dim3(blocks), dim3(256), 0, stream, dst, src, count,
                     bd, per, by_nseg ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_copy_u64(uint64_t *dst, const uint64_t *src, uint64_t count,
                              hipStream_t stream, const BatchDesc *bd, uint32_t per,
                              bool by_nseg) {
  if (count == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(copy_kernel<uint64_t>, dim3(blocks), dim3(256), 0, stream, dst, src, count,
                     bd, per, by_nseg ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherDesc *d, uint32_t nd, uint32_t blocks, uint64_t *count_pool,
                         const uint64_t *gmax_pool, uint64_t *snap, hipStream_t stream) {
  if (nd == 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(blocks), dim3(256), 0, stream, d, nd, count_pool,
                     gmax_pool, snap);
  return hipGetLastError();
}

int wide_blocks_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, wide_kernel<false>, WB, 0) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

template <int BLOCK>
static int sampler_blocks(int &blocks, bool tables) {
  // the fewer of the two variants (one graph, several) a launch of this layout may use
  int b[2] = {0, 0};
  hipError_t e = tables
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[0], sampler_kernel<BLOCK, false, true>, BLOCK, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[0], sampler_kernel<BLOCK, false, false>, BLOCK, 0);
  if (e == hipSuccess)
    e = tables
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[1], sampler_kernel<BLOCK, true, true>, BLOCK, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b[1], sampler_kernel<BLOCK, true, false>, BLOCK, 0);
  blocks = std::min(b[0], b[1]);
  return e == hipSuccess ? 0 : 1;
}

int sampler_blocks_per_cu(int block, bool tables) {
  int blocks = 0, bad = 1;
  if (block == 64) bad = sampler_blocks<64>(blocks, tables);
  else if (block == 128) bad = sampler_blocks<128>(blocks, tables);
  else if (block == 256) bad = sampler_blocks<256>(blocks, tables);
  if (bad) return 1;
  return blocks > 0 ? blocks : 1;
}

}  // namespace kad
