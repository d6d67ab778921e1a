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

constexpr int SAMPLER_BLOCK = 128;  // two waves per sample

struct GraphDev {
  uint32_t n;
  uint64_t arcs;
  const uint32_t *row, *col;   // out-rows
  const uint32_t *rrow, *rcol; // in-rows (alias the out-rows when undirected)
};

// Per-slot working state: one slot per resident sampler workgroup.  Each slot owns
// n tags, n 128-bit path counts (zero between samples), an n-entry list of the
// nodes reached (the frontiers are contiguous segments of it) and a candidate-edge
// buffer of pi_cap entries.
struct SlotState {
  uint32_t slots;
  uint32_t n;
  uint32_t pi_cap;     // power of two
  uint32_t *tag;       // [slots * n]
  uint64_t *sig;       // [slots * n * 2]  (lo, hi)
  uint32_t *visit;     // [slots * n]
  uint64_t *pi;        // [slots * pi_cap]
};

struct SampleOut {
  uint32_t *s, *t, *len, *flags; // [count]
  uint32_t *nodes;               // [count] nodes reached by the two searches
  uint64_t *arcs;                // [count] arcs scanned by level expansions
  uint32_t *path;                // [count * stride], path nodes s..t
  uint32_t stride;
};

// Sample ids [first, first + count) of `phase`, dynamically distributed over the
// slot workgroups through *work (must be 0 at launch).
hipError_t launch_sampler(const GraphDev &g, const SlotState &st, uint64_t seed, uint32_t phase,
                          uint64_t first, uint32_t count, uint32_t *work, const SampleOut &out,
                          uint32_t grid, hipStream_t stream);

// Node tiles of the hit reduction: 8,192 ids each, at most this many tiles (graphs of
// up to 2^25 nodes).
constexpr uint32_t MAX_HIT_TILES_PUBLIC = 4096;
constexpr uint32_t HIT_TILE_IDS = 8192;

// Scratch of the hit reduction: one bin of `cap` node ids per tile (cap >= the hits of
// one call), and the bins' fill counters (all zero between calls).
struct HitScratch {
  uint32_t *bins;
  uint64_t cap;
  uint32_t *bin_count;
};

// count[v] += (or -=, with subtract) the number of samples in [0, nsamp) whose path has
// v as an interior node.  With gmax != NULL also raises gmax[group[v]] to the new count
// of every changed node.
hipError_t launch_hit_reduce(const uint32_t *path, const uint32_t *len, uint32_t stride,
                             uint32_t nsamp, uint32_t n, uint64_t *count, bool subtract,
                             const uint32_t *group, uint64_t *gmax, const HitScratch &hs,
                             hipStream_t stream);

// Zero a small device buffer with a kernel (no memset node when captured).
hipError_t launch_zero_u32(uint32_t *p, uint32_t count, hipStream_t stream);

// Sampler workgroups that fit on the device at once (occupancy query).
int sampler_blocks_per_cu();

}  // namespace kad
