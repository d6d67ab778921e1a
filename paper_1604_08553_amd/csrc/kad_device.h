// Launch interface between the host runtime and the HIP kernels (library-internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kad {

// Tag of a node in a sample's working state: 0 = not reached; the s side stores
// level + 1, the t side stores TAG_T | (level + 1).
constexpr uint32_t TAG_T = 0x80000000u;

constexpr uint32_t FLAG_OVERFLOW = 1u;
constexpr uint32_t FLAG_CAPACITY = 2u;
constexpr uint32_t FLAG_RNG = 4u;

// Launch shape of the sampler: workgroup size (64, 128 or 256 threads, one sample
// per workgroup) and the largest level expansion (in arcs) that takes the combined
// single scan.  Neither changes any result.
struct LaunchShape {
  int block = 128;
  uint32_t small_exp = 128;
};
constexpr int SAMPLER_BLOCKS[3] = {64, 128, 256};

struct GraphDev {
  uint32_t n;
  uint64_t arcs;
  const uint32_t *row, *col;   // out-rows
  const uint32_t *rrow, *rcol; // in-rows (alias the out-rows when undirected)
  uint32_t forward = 0;        // nonzero: always expand the s side (a plain BFS from s)
};

// Per-slot working state: one slot per resident sampler workgroup.  Each slot owns
// n node records of REC_WORDS words -- tag, wide-count position, 128-bit path count
// (low, high) -- all zero between samples, an n-entry list of the nodes reached (the
// frontiers are contiguous segments of it) and a candidate-edge buffer of pi_cap
// entries.  With hbits > 0 (sampler slots only) the n = 2^hbits records of a slot are a
// hash table keyed by node id (word 1 holds id + 1 instead of the wide-count position)
// and vh[j] is the record index of the reached node visit[j].
constexpr uint32_t REC_WORDS = 8;
struct SlotState {
  uint32_t slots;
  uint32_t n;
  uint32_t pi_cap;     // power of two
  uint32_t *rec;       // [slots * n * REC_WORDS]
  uint32_t *visit;     // [slots * n]
  uint64_t *pi;        // [slots * pi_cap]
  uint32_t hbits = 0;  // 0: record v at index v; else log2 of the table size (= n)
  uint32_t *vh = nullptr;  // hashed: [slots * n]
};

// One segment of a multi-query launch: sample ids [first, first + count) of
// (graph, seed, phase), stored at launch indices [begin, begin + count).  Node ids
// written to the path buffer are shifted by id_base (the query's place in a shared
// counter pool), so one hit reduction serves every query of the launch.
struct SampleSeg {
  const uint32_t *row, *col, *rrow, *rcol;
  uint64_t seed;
  uint64_t first;
  uint32_t n;
  uint32_t phase;
  uint32_t begin;
  uint32_t id_base;
  uint32_t wide_only;  // nonzero: sampled by the wide-count kernel only (high diameter)
  uint32_t forward;    // nonzero: the forward search (GraphDev::forward)
};

// Working memory of the wide-count resampling (wide_kernel): the sampler slots' node
// records and node lists are reused (a record's position word holds the node's
// position meanwhile); per wide slot a limb arena and level tables of max_lev levels
// per side.
struct WideState {
  uint32_t slots;       // <= the sampler slots
  uint32_t max_lev;
  uint64_t arena_limbs; // per slot
  uint64_t *arena;      // [slots * arena_limbs]
  uint32_t *lv;         // [slots * 2 * max_lev * 4]
  uint64_t *lbase;      // [slots * 2 * max_lev]
};

// The arguments of one batch in device memory.  A chain of launches recorded once into a
// hipGraph reads them from here on every replay (kernels given a descriptor ignore the
// corresponding arguments): the sampler and the wide-count fix take seed, phase, first,
// count, over segments nseg, and (when nonzero) the path stride; the edge-path rewrite and
// the copies take count (or nseg); the batched hit reduction takes count and the number of
// check intervals niv.
struct BatchDesc {
  uint64_t seed;
  uint64_t first;
  uint32_t count;
  uint32_t phase;
  uint32_t niv;
  uint32_t nseg;
  uint32_t stride;
  uint32_t pad;
};

struct SampleOut {
  uint32_t *s, *t, *len, *flags; // [count]
  uint32_t *nodes;               // [count] nodes reached by the two searches
  uint64_t *arcs;                // [count] arcs scanned by level expansions
  uint32_t *path;                // [count * stride], path nodes s..t
  uint32_t stride;
  // The sampler appends the launch index of every sample it flags FLAG_OVERFLOW or
  // FLAG_CAPACITY (and of every sample of a wide_only segment) to fix_list[0, *fix_count)
  // (room for the launch's samples; *fix_count zero at launch); launch_wide_fix samples
  // them again.  May be null (no list kept).
  uint32_t *fix_list = nullptr;
  uint32_t *fix_count = nullptr;
};

// Sample ids [first, first + count) of `phase`, dynamically distributed over the
// slot workgroups through *work (must be 0 at launch).
// bd (device memory, may be null): the batch's arguments, read by the kernel in place of
// seed, phase, first and count -- the launch is then valid for any batch of at most
// `count` samples.
hipError_t launch_sampler(const GraphDev &g, const SlotState &st, uint64_t seed, uint32_t phase,
                          uint64_t first, uint32_t count, uint32_t *work, const SampleOut &out,
                          uint32_t grid, const LaunchShape &shape, hipStream_t stream,
                          const BatchDesc *bd = nullptr);

// Samples [0, count) of the launch, segment by segment (segs[] in device memory,
// ascending `begin`, segs[0].begin == 0); st.n is the slot capacity (>= every
// segment's n).
hipError_t launch_sampler_multi(const SampleSeg *segs, uint32_t nseg, const SlotState &st,
                                uint32_t count, uint32_t *work, const SampleOut &out,
                                uint32_t grid, const LaunchShape &shape, hipStream_t stream,
                                const BatchDesc *bd = nullptr);

// Sample again, with multi-limb path counts and no limit on the candidate edges but the
// arena, the samples of the launch listed in list[0, *list_count) -- the sampler's fix
// list -- or, with `all` (list == nullptr), every sample of the launch (no sampler launch
// before it).  The results are those of exact arithmetic; FLAG_CAPACITY remains only if
// the arena or the level tables are too small, or the path outgrows the stride; with
// out.fix_list set, such samples are also appended to it (for a launch with larger
// arenas).  work: a counter, zero at launch.  segs == nullptr: the single-graph launch
// (g, seed, phase, first).  With an empty list the kernel's workgroups exit at once.
hipError_t launch_wide_fix(const GraphDev &g, uint64_t seed, uint32_t phase, uint64_t first,
                           const SampleSeg *segs, uint32_t nseg, const SlotState &st,
                           const WideState &ws, uint32_t count, bool all,
                           const uint32_t *list, const uint32_t *list_count, uint32_t *work,
                           const SampleOut &out, hipStream_t stream,
                           const BatchDesc *bd = nullptr);

// Node tiles of the hit reduction: 8,192 ids each, at most this many tiles (graphs of
// up to 2^25 nodes).
constexpr uint32_t MAX_HIT_TILES_PUBLIC = 4096;
constexpr uint32_t HIT_TILE_IDS = 8192;

// Scratch of the hit reduction, in one of two layouts:
//   fixed   (tile_start == nullptr): one bin of `cap` entries per tile, cap >= the
//           hits of one call; one partition pass;
//   compact (tile_start != nullptr): one array of `cap` entries >= the hits of one
//           call, tile t at tile_start[t]; a counting pass and a prefix sum first.
// bin_count and tile_fill hold MAX_HIT_TILES_PUBLIC counters, all zero between calls.
struct HitScratch {
  uint32_t *bins;
  uint64_t cap;
  uint32_t *bin_count;
  uint32_t *tile_start = nullptr;
  uint32_t *tile_fill = nullptr;
};

// count[v] += (or -=, with subtract) the number of samples in [0, nsamp) whose path has
// v as an interior node (v < n: the extent of the counter array).  With gmax != NULL also raises gmax[group[v]] to the new count
// of every changed node.
hipError_t launch_hit_reduce(const uint32_t *path, const uint32_t *len, uint32_t stride,
                             uint32_t nsamp, uint32_t n, uint64_t *count, bool subtract,
                             const uint32_t *group, uint64_t *gmax, const HitScratch &hs,
                             hipStream_t stream);

// Every check interval of a batch in three launches: samples [0, nsamp) in intervals of
// per_iv; count[v] += the interior hits, gmax[group[v]] raised, and snap[i * ngroups + g]
// = group g's largest count after interval i (snap may be coherent pinned host memory).
// tmp: n * (number of intervals) counters and ivmax: (number of intervals) * ngroups,
// both all zero between calls (the kernels leave them so).
hipError_t launch_hit_batch(const uint32_t *path, const uint32_t *len, uint32_t stride,
                            uint32_t nsamp, uint32_t per_iv, uint32_t n, uint64_t *count,
                            const uint32_t *group, uint64_t *gmax, uint32_t ngroups,
                            uint32_t *tmp, uint64_t *ivmax, uint64_t *snap,
                            hipStream_t stream, const BatchDesc *bd = nullptr);

// Edge betweenness: the paths of samples [0, nsamp) (node ids, `stride` apart) rewritten
// as edge ids with a placeholder entry at each end (epath, estride >= stride + 1 apart;
// elen[k] = len[k] + 1, 0 without a path): the node-hit reductions then count every edge
// of every path.  eid: edge id per arc position (nullptr: the position is the id).
hipError_t launch_edge_paths(const uint32_t *path, const uint32_t *len, uint32_t stride,
                             uint32_t nsamp, const uint32_t *row, const uint32_t *col,
                             const uint32_t *eid, uint32_t *epath, uint32_t *elen,
                             uint32_t estride, hipStream_t stream,
                             const BatchDesc *bd = nullptr);

// Zero a device buffer with a kernel (no memset node when captured).
hipError_t launch_zero_u32(uint32_t *p, uint64_t count, hipStream_t stream);
// hist[c] += #{v < n : count[v] == c} for c < bins (hist zeroed by the caller)
hipError_t launch_count_hist(const uint64_t *count, uint32_t n, uint32_t *hist, uint32_t bins,
                             hipStream_t stream);
// group[v] = cgrp[count[v]] for v < n (count[v] < bins)
hipError_t launch_group_map(const uint64_t *count, uint32_t n, const uint32_t *cgrp, uint32_t bins,
                            uint32_t *group, hipStream_t stream);
// dst[i] = src[i], i < count, by a kernel on `stream`; either side may be pinned,
// coherent host memory.  Used instead of runtime copies where a copy must not wait
// behind kernels of other streams, and inside recorded graphs.  With bd the kernel
// copies per * bd->count entries (per * bd->nseg with by_nseg; at most `count`, the
// launch's size).
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, uint64_t count,
                              hipStream_t stream, const BatchDesc *bd = nullptr,
                              uint32_t per = 1, bool by_nseg = false);
hipError_t launch_copy_u64(uint64_t *dst, const uint64_t *src, uint64_t count,
                              hipStream_t stream, const BatchDesc *bd = nullptr,
                              uint32_t per = 1, bool by_nseg = false);
// p[i] = value for i < count.
hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t stream);

// One range copied by launch_gather: snap[dst, dst + len) = src[off, off + len) where src
// is the group-maximum pool (GATHER_GMAX) or the counter pool (GATHER_COUNT; with
// GATHER_COUNT_ZERO the counters are also reset to 0).
enum : uint32_t { GATHER_GMAX = 0, GATHER_COUNT = 1, GATHER_COUNT_ZERO = 2 };
struct GatherDesc {
  uint64_t off;
  uint64_t dst;
  uint32_t len;
  uint32_t mode;
  uint32_t block0;  // first workgroup of this range (ascending over the list)
  uint32_t pad;
};
constexpr uint32_t GATHER_CHUNK = 4096;  // entries per workgroup
// blocks = the sum over descriptors of ceil(len / GATHER_CHUNK).
hipError_t launch_gather(const GatherDesc *d, uint32_t nd, uint32_t blocks, uint64_t *count_pool,
                         const uint64_t *gmax_pool, uint64_t *snap, hipStream_t stream);

// count[v] += 1 for every interior node v (< n) of the paths of samples [0, nsamp), one
// device atomic per hit.
hipError_t launch_hit_add_atomic(const uint32_t *path, const uint32_t *len, uint32_t stride,
                                 uint32_t nsamp, uint32_t n, uint64_t *count,
                                 hipStream_t stream);
// *arcs_total += sum of arcs[0, count); *flags_or |= OR of flags[0, count).
hipError_t launch_sample_sums(const uint64_t *arcs, const uint32_t *flags, uint32_t count,
                              uint64_t *arcs_total, uint32_t *flags_or, hipStream_t stream);

// The fixed working memory of the entry point that allocates nothing: a file-scope device
// array of NOALLOC_SCRATCH_BYTES in the kernels' code object, one copy per device, kept
// until the process ends.  noalloc_scratch gives its device address on the current device
// (looked up once per device with hipGetSymbolAddress).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(void **ptr);

// Sampler workgroups of `block` threads resident per CU (occupancy query).
// Resident sampler workgroups per CU for a workgroup size and slot layout (tables or not).
int sampler_blocks_per_cu(int block, bool tables);
// Wide-count workgroups resident per CU (occupancy query).
int wide_blocks_per_cu();

}  // namespace kad
