// Host-side statistics of the adaptive betweenness algorithm (Borassi & Natale):
// the sample cap omega (Algorithm 1), the vertex diameter it needs, computeDelta
// (Algorithm 2, appendix "How to choose delta_L, delta_U"), the bounds f and g of
// Theorem azuma-borassi, the all-nodes and top-k stopping conditions (section 2,
// Algorithm 3), the top-k half-widths (section 5) and the rank intervals of the
// top-k output.  Binary64 throughout, no FMA contraction, glibc exp/log.
#include "kad_stats.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <condition_variable>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <system_error>
#include <thread>
#include <utility>
#include <vector>

namespace kad {

unsigned parallel_threads(uint32_t n) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  return std::max(1u, std::min({16u, hw, n / 65536u + 1u}));
}

namespace {
// Persistent workers for parallel_ranges (starting threads per call cost about as much as
// the loops they ran).  One job at a time; the calling thread takes share 0.  A share that
// throws does not end its thread: run() rethrows the first exception once every share is
// done.  Threads that cannot be started leave a smaller pool.
class WorkerPool {
 public:
  explicit WorkerPool(unsigned n) {
    for (unsigned i = 1; i < n; ++i) {
      try {
        th_.emplace_back([this, i] { loop(i); });
      } catch (const std::system_error &) {
        break;
      }
    }
  }
  ~WorkerPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      quit_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto &t : th_) t.join();
  }
  unsigned size() const { return (unsigned)th_.size() + 1; }
  void run(unsigned nt, const std::function<void(unsigned)> &job) {
    std::lock_guard<std::mutex> one(run_m_);
    {
      std::lock_guard<std::mutex> lk(m_);
      job_ = &job;
      nt_ = nt;
      left_ = nt - 1;
      ++gen_;
    }
    cv_.notify_all();
    std::exception_ptr err;
    try {
      job(0);
    } catch (...) {
      err = std::current_exception();
    }
    std::unique_lock<std::mutex> lk(m_);
    done_.wait(lk, [&] { return left_ == 0; });
    job_ = nullptr;
    if (!err) err = err_;
    err_ = nullptr;
    lk.unlock();
    if (err) std::rethrow_exception(err);
  }

 private:
  void loop(unsigned i) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(unsigned)> *job = nullptr;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        if (quit_) return;
        if (i >= nt_) continue;
        job = job_;
      }
      std::exception_ptr e;
      try {
        (*job)(i);
      } catch (...) {
        e = std::current_exception();
      }
      std::lock_guard<std::mutex> lk(m_);
      if (e && !err_) err_ = e;
      if (--left_ == 0) done_.notify_one();
    }
  }
  std::vector<std::thread> th_;
  std::mutex m_, run_m_;
  std::condition_variable cv_, done_;
  const std::function<void(unsigned)> *job_ = nullptr;
  std::exception_ptr err_;  // the first exception of a worker's share in the current job
  unsigned nt_ = 0, left_ = 0;
  uint64_t gen_ = 0;
  bool quit_ = false;
};

WorkerPool &workers() {
  static WorkerPool pool(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  return pool;
}
}  // namespace

void parallel_ranges(uint32_t n, const std::function<void(uint32_t, uint32_t, unsigned)> &f) {
  const unsigned nt = std::min(parallel_threads(n), workers().size());
  if (nt == 1) {
    f(0, n, 0);
    return;
  }
  workers().run(nt, [&](unsigned w) {
    const uint32_t b = (uint32_t)((uint64_t)n * w / nt), e = (uint32_t)((uint64_t)n * (w + 1) / nt);
    f(b, e, w);
  });
}

unsigned worker_count() { return workers().size(); }

void parallel_tasks(unsigned tasks, const std::function<void(unsigned)> &f) {
  const unsigned nw = workers().size();
  for (unsigned b = 0; b < tasks; b += nw) {
    const unsigned k = std::min(nw, tasks - b);
    if (k == 1)
      f(b);
    else
      workers().run(k, [&](unsigned w) { f(b + w); });
  }
}

// ------------------------------------------------------------------ schedule

uint64_t omega_of(double epsilon, double delta, uint32_t vd, double c) {
  // floor(log2(VD - 2)) + 1, with VD <= 3 giving 0 + 1
  const uint32_t base = vd > 3 ? vd - 2 : 1u;
  uint32_t fl = 0;
  for (uint32_t x = base; x > 1; x >>= 1) ++fl;
  const double bits = (double)(fl + 1);
  const double value = c / (epsilon * epsilon) * (bits + log(2.0 / delta));
  return (uint64_t)ceil(value);
}

// The cap for edge betweenness: a shortest path has at most VD - 1 edges, and a set of k
// paths shattered by the ranges "paths through edge e" puts each of its paths in 2^(k-1)
// ranges, i.e. on 2^(k-1) of its edges: floor(log2(VD - 1)) + 1 replaces floor(log2(VD - 2)) + 1.
uint64_t omega_edges_of(double epsilon, double delta, uint32_t vd, double c) {
  const uint32_t base = vd > 2 ? vd - 1 : 1u;
  uint32_t fl = 0;
  for (uint32_t x = base; x > 1; x >>= 1) ++fl;
  const double bits = (double)(fl + 1);
  const double value = c / (epsilon * epsilon) * (bits + log(2.0 / delta));
  return (uint64_t)ceil(value);
}

uint64_t alpha_of(uint64_t omega) { return std::max<uint64_t>(1, omega / 100); }

uint64_t interval_of(uint64_t omega) {
  const uint64_t q = omega / 16;
  uint64_t p = 1;
  while (2 * p <= q) p *= 2;
  return std::min<uint64_t>(65536, std::max<uint64_t>(1024, p));
}

// ------------------------------------------------------------------ f and g

double bound_f(double bt, double L, double omega, double tau) {
  // (L/tau) * (a + sqrt(a^2 + x)) with a = 1/3 - omega/tau < 0 and x = 2 bt omega / L,
  // evaluated as (L/tau) * x / (sqrt(a^2 + x) - a), free of cancellation.
  const double a = 1.0 / 3.0 - omega / tau;
  const double x = 2.0 * bt * omega / L;
  return (L / tau) * (x / (sqrt(a * a + x) - a));
}

double bound_g(double bt, double L, double omega, double tau) {
  const double b = 1.0 / 3.0 + omega / tau;
  const double x = 2.0 * bt * omega / L;
  return (L / tau) * (b + sqrt(b * b + x));
}

// ------------------------------------------------------------------ vertex diameter

namespace {

// Distances by BFS from src over rows (rp, cl); only nodes with comp[x] == c when comp
// is given.  Returns the eccentricity (largest finite distance).
uint32_t bfs_farthest(const uint32_t *rp, const uint32_t *cl, uint32_t src,
                      const std::vector<uint32_t> *comp, uint32_t c, std::vector<uint32_t> &dist,
                      std::vector<uint32_t> &queue) {
  size_t head = 0, tail = 0;
  dist[src] = 0;
  queue[tail++] = src;
  uint32_t far = 0;
  while (head < tail) {
    const uint32_t u = queue[head++];
    far = std::max(far, dist[u]);
    for (uint32_t e = rp[u]; e < rp[u + 1]; ++e) {
      const uint32_t x = cl[e];
      if (dist[x] != UINT32_MAX) continue;
      if (comp && (*comp)[x] != c) continue;
      dist[x] = dist[u] + 1;
      queue[tail++] = x;
    }
  }
  for (size_t q = 0; q < tail; ++q) dist[queue[q]] = UINT32_MAX;
  return far;
}

// Level-synchronous BFS from src over rows (rp, cl) through the nodes whose mark is
// `from`, marking each reached node `to` (mark[src] must already be `to`); a large level
// is split over the worker threads, which claim nodes by compare-and-swap on the mark.
// Returns src's eccentricity within those nodes; with root, also the reached node of
// largest degree (the first in id order among equals).
struct BfsScratch {  // reused across the BFS calls of one bound (many components are tiny)
  std::vector<uint32_t> cur, next, lbest, ldeg;
  std::vector<std::vector<uint32_t>> local;
};

uint32_t bfs_levels(const uint32_t *rp, const uint32_t *cl, uint32_t src, uint32_t *mark,
                    uint32_t from, uint32_t to, uint32_t *root, BfsScratch &sc) {
  constexpr size_t PAR_MIN = 8192;  // frontier nodes below which a level runs on one thread
  std::vector<uint32_t> &cur = sc.cur, &next = sc.next;
  cur.assign(1, src);
  uint32_t best = src, best_deg = rp[src + 1] - rp[src], ecc = 0;
  auto better = [](uint32_t d, uint32_t v, uint32_t bd, uint32_t bv) {
    return d > bd || (d == bd && v < bv);
  };
  const unsigned nw = (unsigned)workers().size();
  sc.local.resize(nw);
  sc.lbest.resize(nw);
  sc.ldeg.resize(nw);
  std::vector<std::vector<uint32_t>> &local = sc.local;
  std::vector<uint32_t> &lbest = sc.lbest, &ldeg = sc.ldeg;
  for (;;) {
    next.clear();
    if (cur.size() < PAR_MIN || nw == 1) {
      for (const uint32_t u : cur)
        for (uint32_t e = rp[u]; e < rp[u + 1]; ++e) {
          const uint32_t x = cl[e];
          if (mark[x] != from) continue;
          mark[x] = to;
          next.push_back(x);
          const uint32_t d = rp[x + 1] - rp[x];
          if (root && better(d, x, best_deg, best)) {
            best = x;
            best_deg = d;
          }
        }
    } else {
      const unsigned nt = (unsigned)std::min<size_t>(nw, cur.size() / (PAR_MIN / 8));
      workers().run(nt, [&](unsigned w) {
        std::vector<uint32_t> &out = local[w];
        out.clear();
        uint32_t b = UINT32_MAX, bd = 0;
        const size_t lo = cur.size() * w / nt, hi = cur.size() * (w + 1) / nt;
        for (size_t q = lo; q < hi; ++q) {
          const uint32_t u = cur[q];
          for (uint32_t e = rp[u]; e < rp[u + 1]; ++e) {
            const uint32_t x = cl[e];
            uint32_t expect = from;
            if (__atomic_load_n(&mark[x], __ATOMIC_RELAXED) != from ||
                !__atomic_compare_exchange_n(&mark[x], &expect, to, false, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED))
              continue;
            out.push_back(x);
            const uint32_t d = rp[x + 1] - rp[x];
            if (b == UINT32_MAX || better(d, x, bd, b)) {
              b = x;
              bd = d;
            }
          }
        }
        lbest[w] = b;
        ldeg[w] = bd;
      });
      for (unsigned w = 0; w < nt; ++w) {
        next.insert(next.end(), local[w].begin(), local[w].end());
        if (root && lbest[w] != UINT32_MAX && better(ldeg[w], lbest[w], best_deg, best)) {
          best = lbest[w];
          best_deg = ldeg[w];
        }
      }
    }
    if (next.empty()) break;
    ++ecc;
    cur.swap(next);
  }
  if (root) *root = best;
  return ecc;
}

// Undirected graphs: the strongly connected components are the connected components and
// no arc joins two of them, so the bound below is the largest 2 ecc(r_C) + 1 over the
// components C (r_C: C's node of largest degree, the first in id order among equals; an
// isolated node gives 1).  One BFS labels a component and finds r_C, a second measures
// ecc(r_C).  The node of largest degree in the whole graph (the first in id order among
// equals) is r_C of its own component, the giant one of a sparse power-law graph, so that
// component goes first and takes a single BFS from it.
uint32_t vd_undirected(uint32_t n, const uint32_t *row, const uint32_t *col) {
  std::vector<uint32_t> mark(n, 0);  // 0 unseen, 1 labelled, 2 measured
  BfsScratch sc;
  uint64_t answer = 0;
  uint32_t p = 0;
  for (uint32_t v = 1; v < n; ++v)
    if (row[v + 1] - row[v] > row[p + 1] - row[p]) p = v;
  if (row[p + 1] > row[p]) {
    mark[p] = 2;
    answer = 2ull * bfs_levels(row, col, p, mark.data(), 0, 2, nullptr, sc) + 1;
  }
  for (uint32_t v = 0; v < n; ++v) {
    if (mark[v] != 0) continue;
    if (row[v + 1] == row[v]) {
      mark[v] = 2;
      answer = std::max<uint64_t>(answer, 1);
      continue;
    }
    uint32_t root = v;
    mark[v] = 1;
    (void)bfs_levels(row, col, v, mark.data(), 0, 1, &root, sc);
    mark[root] = 2;
    const uint32_t ecc = bfs_levels(row, col, root, mark.data(), 1, 2, nullptr, sc);
    answer = std::max<uint64_t>(answer, 2ull * ecc + 1);
  }
  return (uint32_t)std::min<uint64_t>(answer, UINT32_MAX);
}

// Strongly connected components by Tarjan's algorithm (iterative), with one component
// known beforehand contracted into a single node: the nodes with mark[v] == gmark form a
// strongly connected component represented by g, and gout lists the heads of its arcs that
// leave it.  An arc into that component leads to g, and its other nodes are not visited
// (they take g's number on return).  Contracting a strongly connected component leaves
// the condensation as it was, so components are still numbered in the order Tarjan
// completes them, a reverse topological order of the condensation: every arc u->x
// between components has comp[u] > comp[x].
uint32_t tarjan_scc(uint32_t n, const uint32_t *row, const uint32_t *col, const uint32_t *mark,
                    uint32_t gmark, uint32_t g, const std::vector<uint32_t> &gout,
                    std::vector<uint32_t> &comp) {
  std::vector<uint32_t> index(n, UINT32_MAX), low(n, 0), stack, call;
  std::vector<std::pair<const uint32_t *, const uint32_t *>> next;  // arcs left, per call
  std::vector<uint8_t> on_stack(n, 0);
  comp.assign(n, UINT32_MAX);
  uint32_t next_index = 0, ncomp = 0;
  auto open = [&](uint32_t u) {
    index[u] = low[u] = next_index++;
    stack.push_back(u);
    on_stack[u] = 1;
    call.push_back(u);
    if (u == g)
      next.emplace_back(gout.data(), gout.data() + gout.size());
    else
      next.emplace_back(col + row[u], col + row[u + 1]);
  };
  for (uint32_t root = 0; root < n; ++root) {
    if (index[root] != UINT32_MAX || (mark[root] == gmark && root != g)) continue;
    open(root);
    while (!call.empty()) {
      const uint32_t u = call.back();
      if (next.back().first != next.back().second) {
        uint32_t x = *next.back().first++;
        if (mark[x] == gmark) x = g;
        if (index[x] == UINT32_MAX)
          open(x);
        else if (on_stack[x])
          low[u] = std::min(low[u], index[x]);
        continue;
      }
      if (low[u] == index[u]) {
        uint32_t x;
        do {
          x = stack.back();
          stack.pop_back();
          on_stack[x] = 0;
          comp[x] = ncomp;
        } while (x != u);
        ++ncomp;
      }
      call.pop_back();
      next.pop_back();
      if (!call.empty()) low[call.back()] = std::min(low[call.back()], low[u]);
    }
  }
  for (uint32_t v = 0; v < n; ++v)
    if (mark[v] == gmark) comp[v] = comp[g];
  return ncomp;
}

// Directed graphs: the bound over the condensation, weight(C) = ecc_out_C(r_C) +
// ecc_in_C(r_C) + 1 (r_C: C's node of largest total degree, the first in id order among
// equals), summed along the heaviest chain of components.  The node p of largest total
// degree in the whole graph is r_C of its own component G, which in a sparse power-law
// graph is the giant one; G and its weight come from three BFS from p, run level by level
// on the worker threads, and Tarjan's algorithm then walks only the rest:
//  1. forward over all nodes: the nodes p reaches;
//  2. backward through those nodes only: the ones that also reach p, which is G (every
//     node on a path from a node of G to p is in G).  A shortest path between two nodes
//     of G never leaves G, so this BFS's depth is ecc_in_G(p);
//  3. forward through G: ecc_out_G(p).
uint32_t vd_directed(uint32_t n, const uint32_t *row, const uint32_t *col, const uint32_t *rrow,
                     const uint32_t *rcol) {
  auto degree = [&](uint32_t v) {
    return (uint64_t)(row[v + 1] - row[v]) + (rrow[v + 1] - rrow[v]);
  };
  uint32_t p = 0;
  for (uint32_t v = 1; v < n; ++v)
    if (degree(v) > degree(p)) p = v;
  constexpr uint32_t IN_G = 3;  // marks: 0 unseen, 1 reached from p, 2 and 3 in G
  std::vector<uint32_t> mark(n, 0);
  BfsScratch sc;
  mark[p] = 1;
  (void)bfs_levels(row, col, p, mark.data(), 0, 1, nullptr, sc);
  mark[p] = 2;
  const uint32_t ecc_in = bfs_levels(rrow, rcol, p, mark.data(), 1, 2, nullptr, sc);
  mark[p] = IN_G;
  const uint32_t ecc_out = bfs_levels(row, col, p, mark.data(), 2, IN_G, nullptr, sc);
  // heads of the arcs that leave G, gathered over ranges of tails on the worker threads
  std::vector<std::vector<uint32_t>> part(workers().size());
  parallel_ranges(n, [&](uint32_t lo, uint32_t hi, unsigned w) {
    std::vector<uint32_t> &out = part[w];
    out.clear();
    for (uint32_t v = lo; v < hi; ++v) {
      if (mark[v] != IN_G) continue;
      for (uint32_t e = row[v]; e < row[v + 1]; ++e)
        if (mark[col[e]] != IN_G) out.push_back(col[e]);
    }
  });
  std::vector<uint32_t> gout;
  for (auto &pv : part) gout.insert(gout.end(), pv.begin(), pv.end());

  std::vector<uint32_t> comp;
  const uint32_t nc = tarjan_scc(n, row, col, mark.data(), IN_G, p, gout, comp);
  const uint32_t cg = comp[p];
  std::vector<uint32_t> root(nc, UINT32_MAX);
  for (uint32_t v = 0; v < n; ++v) {
    const uint32_t c = comp[v];
    if (root[c] == UINT32_MAX || degree(v) > degree(root[c])) root[c] = v;
  }
  // members of each component, ids ascending (a counting pass; most components of a
  // sparse directed graph are single nodes)
  std::vector<uint32_t> mstart(nc + 1, 0), member(n);
  for (uint32_t v = 0; v < n; ++v) mstart[comp[v] + 1]++;
  for (uint32_t c = 0; c < nc; ++c) mstart[c + 1] += mstart[c];
  {
    std::vector<uint32_t> fill(mstart.begin(), mstart.end() - 1);
    for (uint32_t v = 0; v < n; ++v) member[fill[comp[v]]++] = v;
  }
  std::vector<uint32_t> dist(n, UINT32_MAX), queue(n);
  std::vector<uint64_t> weight(nc);
  for (uint32_t c = 0; c < nc; ++c) {
    if (c == cg) {  // r_G is p: no node has a larger degree, none before p an equal one
      weight[c] = (uint64_t)ecc_out + ecc_in + 1;
    } else if (mstart[c + 1] - mstart[c] == 1) {  // a single node: both eccentricities 0
      weight[c] = 1;
    } else {
      weight[c] = (uint64_t)bfs_farthest(row, col, root[c], &comp, c, dist, queue) +
                  bfs_farthest(rrow, rcol, root[c], &comp, c, dist, queue) + 1;
    }
  }
  // Tarjan numbering is reverse topological: process components from the highest id
  // (sources) down; heaviest[c] = weight[c] + max over arcs into c.
  std::vector<uint64_t> heaviest(nc, 0);
  uint64_t answer = 0;
  auto best_into = [&](uint32_t c, uint32_t lo, uint32_t hi) {
    uint64_t best = 0;
    for (uint32_t i = lo; i < hi; ++i)
      for (uint32_t v = member[i], e = rrow[v]; e < rrow[v + 1]; ++e) {
        const uint32_t c2 = comp[rcol[e]];
        if (c2 != c) best = std::max(best, heaviest[c2]);
      }
    return best;
  };
  for (uint32_t c = nc; c-- > 0;) {
    uint64_t in_best = 0;
    if (c == cg) {  // G's members over the worker threads (their arcs are most of the graph)
      std::vector<uint64_t> part_best(workers().size(), 0);
      parallel_ranges(mstart[c + 1] - mstart[c], [&](uint32_t lo, uint32_t hi, unsigned w) {
        part_best[w] = best_into(c, mstart[c] + lo, mstart[c] + hi);
      });
      in_best = *std::max_element(part_best.begin(), part_best.end());
    } else {
      in_best = best_into(c, mstart[c], mstart[c + 1]);
    }
    heaviest[c] = in_best + weight[c];
    answer = std::max(answer, heaviest[c]);
  }
  return (uint32_t)std::min<uint64_t>(answer, UINT32_MAX);
}

}  // namespace

int vertex_diameter(uint32_t n, uint64_t arcs, const uint32_t *row, const uint32_t *col,
                    const uint32_t *rrow, const uint32_t *rcol, double exact_limit, uint32_t *vd,
                    bool *exact) {
  if (n == 0 || !row || !rrow || (arcs && (!col || !rcol))) return -1;
  if ((double)n * (double)arcs <= exact_limit) {
    // exact: the largest BFS eccentricity over all sources, plus one node (sources dealt
    // out over the worker threads)
    const unsigned nt = worker_count();
    std::vector<uint32_t> best(nt, 0);
    parallel_tasks(nt, [&](unsigned w) {
      std::vector<uint32_t> dist(n, UINT32_MAX), queue(n);
      for (uint32_t s = w; s < n; s += nt)
        best[w] = std::max(best[w], bfs_farthest(row, col, s, nullptr, 0, dist, queue));
    });
    *vd = *std::max_element(best.begin(), best.end()) + 1;
    *exact = true;
    return 0;
  }
  // bound over the condensation: weight(C) = ecc_out_C(r) + ecc_in_C(r) + 1
  if (rrow == row && rcol == col) {  // undirected: the same bound, component by component
    *vd = vd_undirected(n, row, col);
    *exact = false;
    return 0;
  }
  *vd = vd_directed(n, row, col, rrow, rcol);
  *exact = false;
  return 0;
}

// ------------------------------------------------------------------ computeDelta

namespace {
// Open-addressing map from a double's bit pattern to a slot index (values repeat a lot:
// a node's constant depends only on its pilot count and its wanted half-widths).
class ValueIndex {
 public:
  explicit ValueIndex(size_t expect) {
    size_t cap = 1024;
    while (cap < 2 * expect) cap *= 2;
    keys_.assign(cap, EMPTY);
    slot_.assign(cap, 0);
  }
  // index of x among the distinct values, inserting it (with the next index) if new
  uint32_t find_or_add(double x) {
    uint64_t k;
    memcpy(&k, &x, 8);
    if (k == EMPTY) k = EMPTY_ALIAS;
    size_t h = (size_t)((k * 0x9E3779B97F4A7C15ULL) >> 17) & (keys_.size() - 1);
    while (true) {
      if (keys_[h] == k) return slot_[h];
      if (keys_[h] == EMPTY) {
        keys_[h] = k;
        slot_[h] = (uint32_t)values.size();
        values.push_back(x);
        if (2 * values.size() > keys_.size()) grow();
        return (uint32_t)values.size() - 1;
      }
      h = (h + 1) & (keys_.size() - 1);
    }
  }
  std::vector<double> values;

 private:
  static constexpr uint64_t EMPTY = ~0ULL;                  // a NaN pattern, never a constant
  static constexpr uint64_t EMPTY_ALIAS = 0xFFF8000000000001ULL;
  void grow() {
    std::vector<uint64_t> old_k;
    std::vector<uint32_t> old_s;
    old_k.swap(keys_);
    old_s.swap(slot_);
    keys_.assign(old_k.size() * 2, EMPTY);
    slot_.assign(old_k.size() * 2, 0);
    for (size_t q = 0; q < old_k.size(); ++q) {
      if (old_k[q] == EMPTY) continue;
      size_t h = (size_t)((old_k[q] * 0x9E3779B97F4A7C15ULL) >> 17) & (keys_.size() - 1);
      while (keys_[h] != EMPTY) h = (h + 1) & (keys_.size() - 1);
      keys_[h] = old_k[q];
      slot_[h] = old_s[q];
    }
  }
  std::vector<uint64_t> keys_;
  std::vector<uint32_t> slot_;
};
}  // namespace

namespace {
// The constants c = 2 b0 omega / lambda^2 of the nodes, as distinct values with
// multiplicities, and the bisection for C over them: the smallest C with
// sum_v exp(-C/c_L(v)) + exp(-C/c_U(v)) <= delta/2 - eps_bal*delta (the sum decreases in
// C).  Lq[q] = L of distinct value q.
struct DeltaSolver {
  ValueIndex index{4096};
  std::vector<double> mult;
  uint32_t add_value(double x, double times) {
    const uint32_t q = index.find_or_add(x);
    if (mult.size() < index.values.size()) mult.resize(index.values.size(), 0.0);
    mult[q] += times;
    return q;
  }
  void solve(uint32_t n, double delta, double eps_bal, std::vector<double> &Lq, double *C_out) {
    const size_t nd = index.values.size();
    if (mult.size() < nd) mult.resize(nd, 0.0);
    std::vector<uint32_t> ord(nd);
    for (uint32_t q = 0; q < nd; ++q) ord[q] = q;
    std::sort(ord.begin(), ord.end(),
              [&](uint32_t a, uint32_t b) { return index.values[a] < index.values[b]; });
    auto term = [](double C, double c) { return c == 0.0 ? 0.0 : exp(-C / c); };
    auto total = [&](double C) {
      double s = 0.0;
      for (uint32_t q : ord) s += mult[q] * term(C, index.values[q]);
      return s;
    };
    const double target = delta / 2.0 - eps_bal * delta;
    double lo = 0.0, hi = 1.0;
    while (total(hi) > target) hi *= 2.0;
    for (int it = 0; it < 100; ++it) {
      const double mid = (lo + hi) / 2.0;
      if (total(mid) > target)
        lo = mid;
      else
        hi = mid;
    }
    const double C = hi;
    const double floor_add = eps_bal * delta / (2.0 * (double)n);
    Lq.resize(nd);
    for (size_t q = 0; q < nd; ++q) Lq[q] = -log(term(C, index.values[q]) + floor_add);
    if (C_out) *C_out = C;
  }
};

// Uniform half-widths: the constants of the nodes with pilot count c, for every count
// present (h[c] > 0) in ascending order; group = rank of the count among those present.
void uniform_values(DeltaSolver &S, const uint64_t *h, uint64_t cmax, uint64_t alpha,
                    uint64_t omega, double lam_l, double lam_u, std::vector<uint32_t> &ca,
                    std::vector<uint32_t> &cb, std::vector<uint32_t> &cgrp, uint32_t &ngrp) {
  ca.assign(cmax + 1, 0);
  cb.assign(cmax + 1, 0);
  cgrp.assign(cmax + 1, 0);
  ngrp = 0;
  for (uint64_t c = 0; c <= cmax; ++c) {
    if (!h[c]) continue;
    const double b0 = (double)c / (double)alpha;
    ca[c] = S.add_value(2.0 * b0 * (double)omega / (lam_l * lam_l), (double)h[c]);
    cb[c] = S.add_value(2.0 * b0 * (double)omega / (lam_u * lam_u), (double)h[c]);
    cgrp[c] = ngrp++;
  }
}
}  // namespace

void compute_delta(uint32_t n, const uint64_t *count0, uint64_t alpha, uint64_t omega,
                   const double *lam_l, const double *lam_u, double delta, double eps_bal,
                   double *L_l, double *L_u, double *C_out, Groups *groups) {
  // The 2n constants c_L(v) = 2 b0(v) omega / lambda_L(v)^2 (and c_U) are handled as
  // indices into their distinct values with multiplicities.
  DeltaSolver S;
  // Uniform half-widths (the all-nodes task): a node's constants depend on its pilot
  // count only, so they are computed once per distinct count.
  const unsigned nt = parallel_threads(n);
  std::vector<uint8_t> t_uniform(nt, 1);
  std::vector<uint64_t> t_cmax(nt, 0);
  parallel_ranges(n, [&](uint32_t b0, uint32_t e0, unsigned w) {
    uint64_t cm = 0;
    bool un = true;
    for (uint32_t v = b0; v < e0; ++v) {
      un = un && lam_l[v] == lam_l[0] && lam_u[v] == lam_u[0];
      cm = std::max(cm, count0[v]);
    }
    t_uniform[w] = un;
    t_cmax[w] = cm;
  });
  const bool uniform = std::all_of(t_uniform.begin(), t_uniform.end(), [](uint8_t x) { return x; });
  const uint64_t cmax = *std::max_element(t_cmax.begin(), t_cmax.end());
  std::vector<uint32_t> il, iu;        // general path: per-node value indices
  std::vector<std::pair<uint32_t, uint32_t>> gpairs_out;  // general path: group -> (il, iu)
  std::vector<uint32_t> ca, cb, cgrp;  // uniform path: per-count value indices and group
  if (uniform && cmax < (1u << 24)) {
    std::vector<std::vector<uint32_t>> th(nt, std::vector<uint32_t>(cmax + 1, 0));
    parallel_ranges(n, [&](uint32_t b0, uint32_t e0, unsigned w) {
      for (uint32_t v = b0; v < e0; ++v) th[w][count0[v]]++;
    });
    std::vector<uint64_t> h(cmax + 1, 0);
    for (uint64_t c = 0; c <= cmax; ++c)
      for (unsigned w = 0; w < nt; ++w) h[c] += th[w][c];
    uint32_t ngrp = 0;
    uniform_values(S, h.data(), cmax, alpha, omega, lam_l[0], lam_u[0], ca, cb, cgrp, ngrp);
    if (groups) {
      groups->L_l.assign(ngrp, 0.0);
      groups->L_u.assign(ngrp, 0.0);
    }
  } else {
    // Most nodes repeat an earlier (count0, lambda_l, lambda_u): a direct-mapped memo of
    // that triple skips recomputing the same two constants.  Ranges of nodes on the worker
    // threads number their distinct constants (and groups) in order of first appearance;
    // merged in range order, the numbering is the one a single pass over the nodes gives,
    // and the multiplicities are whole counts.
    il.resize(n);
    iu.resize(n);
    struct Memo {
      uint64_t c0, ll, lu;
      uint32_t a, b;
      bool used;
    };
    const unsigned nw = workers().size();
    std::vector<std::unique_ptr<ValueIndex>> loc(nw);
    std::vector<std::vector<uint64_t>> lmult(nw);
    std::vector<uint8_t> ran(nw, 0);
    parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
      ran[w] = 1;
      loc[w].reset(new ValueIndex(1024));
      ValueIndex &X = *loc[w];
      std::vector<uint64_t> &lm = lmult[w];
      lm.clear();
      std::vector<Memo> memo(4096, Memo{0, 0, 0, 0, 0, false});
      for (uint32_t v = vb; v < ve; ++v) {
        uint64_t bl, bu;
        memcpy(&bl, &lam_l[v], 8);
        memcpy(&bu, &lam_u[v], 8);
        const uint64_t h = (count0[v] * 0x9E3779B97F4A7C15ULL) ^ (bl * 0xC2B2AE3D27D4EB4FULL) ^
                           (bu * 0x165667B19E3779F9ULL);
        Memo &m = memo[(h >> 40) & 4095];
        if (!(m.used && m.c0 == count0[v] && m.ll == bl && m.lu == bu)) {
          const double b0 = (double)count0[v] / (double)alpha;
          const double cl = 2.0 * b0 * (double)omega / (lam_l[v] * lam_l[v]);
          const double cu = 2.0 * b0 * (double)omega / (lam_u[v] * lam_u[v]);
          m = Memo{count0[v], bl, bu, X.find_or_add(cl), X.find_or_add(cu), true};
          if (lm.size() < X.values.size()) lm.resize(X.values.size(), 0);
        }
        il[v] = m.a;
        iu[v] = m.b;
        lm[m.a]++;
        lm[m.b]++;
      }
    });
    std::vector<std::vector<uint32_t>> remap(nw);
    for (unsigned w = 0; w < nw; ++w) {
      if (!ran[w]) continue;
      const std::vector<double> &vals = loc[w]->values;
      remap[w].resize(vals.size());
      for (size_t q = 0; q < vals.size(); ++q) {
        const uint32_t g = S.index.find_or_add(vals[q]);
        if (S.mult.size() < S.index.values.size()) S.mult.resize(S.index.values.size(), 0.0);
        S.mult[g] += (double)lmult[w][q];
        remap[w][q] = g;
      }
    }
    parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
      const std::vector<uint32_t> &r = remap[w];
      for (uint32_t v = vb; v < ve; ++v) {
        il[v] = r[il[v]];
        iu[v] = r[iu[v]];
      }
    });
    if (groups) {  // group = distinct (il, iu) pair, numbered by first appearance
      struct GMemo {  // most nodes repeat an earlier pair: a direct-mapped memo before the map
        uint32_t a, b, g;
        bool used;
      };
      std::vector<std::vector<std::pair<uint32_t, uint32_t>>> lpairs(nw);
      groups->of.resize(n);
      parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
        std::map<std::pair<uint32_t, uint32_t>, uint32_t> ids;
        std::vector<std::pair<uint32_t, uint32_t>> &lp = lpairs[w];
        lp.clear();
        std::vector<GMemo> gm(4096, GMemo{0, 0, 0, false});
        for (uint32_t v = vb; v < ve; ++v) {
          GMemo &m = gm[((il[v] * 0x9E3779B1u) ^ (iu[v] * 0x85EBCA6Bu)) >> 20];
          if (!(m.used && m.a == il[v] && m.b == iu[v])) {
            const auto key = std::make_pair(il[v], iu[v]);
            auto it = ids.find(key);
            if (it == ids.end()) {
              it = ids.emplace(key, (uint32_t)lp.size()).first;
              lp.push_back(key);
            }
            m = GMemo{il[v], iu[v], it->second, true};
          }
          groups->of[v] = m.g;
        }
      });
      std::map<std::pair<uint32_t, uint32_t>, uint32_t> gids;
      std::vector<std::pair<uint32_t, uint32_t>> gpairs;  // group id -> (il, iu)
      std::vector<std::vector<uint32_t>> gremap(nw);
      for (unsigned w = 0; w < nw; ++w) {
        if (!ran[w]) continue;
        for (const auto &key : lpairs[w]) {
          auto it = gids.find(key);
          if (it == gids.end()) {
            it = gids.emplace(key, (uint32_t)gpairs.size()).first;
            gpairs.push_back(key);
          }
          gremap[w].push_back(it->second);
        }
      }
      parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
        const std::vector<uint32_t> &r = gremap[w];
        for (uint32_t v = vb; v < ve; ++v) groups->of[v] = r[groups->of[v]];
      });
      groups->L_l.assign(gpairs.size(), 0.0);
      groups->L_u.assign(gpairs.size(), 0.0);
      gpairs_out = std::move(gpairs);
    }
  }
  std::vector<double> Lq;
  S.solve(n, delta, eps_bal, Lq, C_out);
  if (!ca.empty()) {
    if (groups) {
      groups->of.resize(n);
      for (uint64_t c = 0; c <= cmax; ++c) {
        groups->L_l[cgrp[c]] = Lq[ca[c]];
        groups->L_u[cgrp[c]] = Lq[cb[c]];
      }
    }
    parallel_ranges(n, [&](uint32_t b0, uint32_t e0, unsigned) {
      for (uint32_t v = b0; v < e0; ++v) {
        const uint64_t c = count0[v];
        L_l[v] = Lq[ca[c]];
        L_u[v] = Lq[cb[c]];
        if (groups) groups->of[v] = cgrp[c];
      }
    });
  } else {
    parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned) {
      for (uint32_t v = vb; v < ve; ++v) {
        L_l[v] = Lq[il[v]];
        L_u[v] = Lq[iu[v]];
      }
    });
    if (groups)  // every node of a group has its pair's values
      for (size_t g = 0; g < gpairs_out.size(); ++g) {
        groups->L_l[g] = Lq[gpairs_out[g].first];
        groups->L_u[g] = Lq[gpairs_out[g].second];
      }
  }
}

void compute_delta_hist(uint32_t n, const uint64_t *hist, uint64_t cmax, uint64_t alpha,
                        uint64_t omega, double lam_l, double lam_u, double delta, double eps_bal,
                        std::vector<uint32_t> &cgrp, Groups &groups, double *C_out) {
  DeltaSolver S;
  std::vector<uint32_t> ca, cb;
  uint32_t ngrp = 0;
  uniform_values(S, hist, cmax, alpha, omega, lam_l, lam_u, ca, cb, cgrp, ngrp);
  std::vector<double> Lq;
  S.solve(n, delta, eps_bal, Lq, C_out);
  groups.of.clear();
  groups.L_l.assign(ngrp, 0.0);
  groups.L_u.assign(ngrp, 0.0);
  for (uint64_t c = 0; c <= cmax; ++c) {
    if (!hist[c]) continue;
    groups.L_l[cgrp[c]] = Lq[ca[c]];
    groups.L_u[cgrp[c]] = Lq[cb[c]];
  }
}

// ------------------------------------------------------------------ top-k half-widths

namespace {
// nodes by count descending, id ascending.  Pilot counts are at most alpha: placed by a
// counting pass (ids ascending within a count), O(n + largest count) instead of a sort.
void estimate_order(uint32_t n, const uint64_t *count, std::vector<uint32_t> &ord) {
  ord.resize(n);
  uint64_t cmax = 0;
  for (uint32_t v = 0; v < n; ++v) cmax = std::max(cmax, count[v]);
  if (cmax < (1ull << 26)) {
    std::vector<uint32_t> pos(cmax + 2, 0);  // bucket cmax - c holds count c
    for (uint32_t v = 0; v < n; ++v) pos[cmax - count[v] + 1]++;
    for (uint64_t b = 1; b <= cmax + 1; ++b) pos[b] += pos[b - 1];
    for (uint32_t v = 0; v < n; ++v) ord[pos[cmax - count[v]]++] = v;
    return;
  }
  for (uint32_t v = 0; v < n; ++v) ord[v] = v;
  std::sort(ord.begin(), ord.end(), [count](uint32_t a, uint32_t b) {
    return count[a] != count[b] ? count[a] > count[b] : a < b;
  });
}
double clamp_unit(double x, double eps) { return std::min(1.0, std::max(eps, x)); }

// The first m nodes in the order of count descending, id ascending.  For small m each
// range of nodes on the worker threads keeps its m first and the m first of those are
// taken (the order is total, so they are the same nodes); otherwise the full order.
void head_by_count(uint32_t n, const uint64_t *count, uint32_t m, std::vector<uint32_t> &head) {
  auto cmp = [count](uint32_t a, uint32_t b) {
    return count[a] != count[b] ? count[a] > count[b] : a < b;
  };
  if ((uint64_t)m * 8 > n || parallel_threads(n) == 1) {
    estimate_order(n, count, head);
    head.resize(m);
    return;
  }
  std::vector<std::vector<uint32_t>> part(workers().size());
  parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned w) {
    std::vector<uint32_t> &p = part[w];
    p.resize(ve - vb);
    for (uint32_t v = vb; v < ve; ++v) p[v - vb] = v;
    if (p.size() > m) {
      std::nth_element(p.begin(), p.begin() + (m - 1), p.end(), cmp);
      p.resize(m);
    }
  });
  head.clear();
  for (auto &p : part) head.insert(head.end(), p.begin(), p.end());
  std::nth_element(head.begin(), head.begin() + (m - 1), head.end(), cmp);
  head.resize(m);
  std::sort(head.begin(), head.end(), cmp);
}
}  // namespace

// Section 5's half-widths: the k nodes of largest pilot count get theirs from the gaps to
// their neighbours in that order (eps where two of the first k+1 lie within 2 eps); every
// other node has lambda_L = 1 and lambda_U from the gap below the k-th node's lower end.
// Only the first k+1 positions of the order matter, so only they are found; the others'
// values depend on their own count alone and are written on the worker threads.
void topk_lambdas(uint32_t n, uint32_t k, const uint64_t *count0, uint64_t alpha, double eps,
                  double *lam_l, double *lam_u) {
  const uint32_t m = (uint32_t)std::min<uint64_t>(n, (uint64_t)k + 1);
  std::vector<uint32_t> ord;  // positions 0..m-1 of the order
  head_by_count(n, count0, m, ord);
  const double A = (double)alpha;
  auto b0 = [&](uint32_t pos) { return (double)count0[ord[pos]] / A; };
  std::vector<uint8_t> tie(m, 0);
  for (uint32_t i = 0; i < k; ++i)
    if (i + 1 < n && b0(i) - b0(i + 1) < 2.0 * eps) tie[i] = tie[i + 1] = 1;
  std::vector<double> top_l(k), top_u(k);
  for (uint32_t i = 0; i < k; ++i) {
    double up = i == 0 ? 1.0 : (b0(i - 1) - b0(i)) / 2.0;
    double dn = i + 1 < n ? (b0(i) - b0(i + 1)) / 2.0 : 1.0;
    if (tie[i]) up = dn = eps;
    top_u[i] = clamp_unit(up, eps);
    top_l[i] = clamp_unit(dn, eps);
  }
  const double kth_low = b0(k - 1) - top_l[k - 1];
  parallel_ranges(n, [&](uint32_t vb, uint32_t ve, unsigned) {
    for (uint32_t v = vb; v < ve; ++v) {
      lam_l[v] = 1.0;
      lam_u[v] = clamp_unit(kth_low - (double)count0[v] / A, eps);
    }
  });
  for (uint32_t i = 0; i < k; ++i) {
    lam_l[ord[i]] = top_l[i];
    lam_u[ord[i]] = top_u[i];
  }
  if (k < n && tie[k]) lam_l[ord[k]] = lam_u[ord[k]] = eps;
}

// ------------------------------------------------------------------ stopping conditions

StopChecker::StopChecker(uint32_t n, uint32_t mode, uint32_t k, double eps, uint64_t omega,
                         const double *L_l, const double *L_u)
    : n_(n), mode_(mode), k_(k), eps_(eps), omega_(omega), Ll_(L_l), Lu_(L_u) {
  // group = distinct (L_l, L_u) pair (a direct-mapped memo in front of the map: most
  // nodes repeat an earlier pair)
  std::map<std::pair<uint64_t, uint64_t>, uint32_t> ids;
  struct Memo {
    uint64_t a, b;
    uint32_t g;
    bool used;
  };
  std::vector<Memo> memo(4096, Memo{0, 0, 0, false});
  group_.resize(n);
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t a, b;
    memcpy(&a, &L_l[v], 8);
    memcpy(&b, &L_u[v], 8);
    Memo &m = memo[((a * 0x9E3779B97F4A7C15ULL ^ b * 0xC2B2AE3D27D4EB4FULL) >> 40) & 4095];
    if (!(m.used && m.a == a && m.b == b)) {
      auto key = std::make_pair(a, b);
      auto it = ids.find(key);
      if (it == ids.end()) {
        it = ids.emplace(key, (uint32_t)gL_l_.size()).first;
        gL_l_.push_back(L_l[v]);
        gL_u_.push_back(L_u[v]);
      }
      m = Memo{a, b, it->second, true};
    }
    group_[v] = m.g;
  }
  gmax_.resize(gL_l_.size());
  if (mode_ == 1) in_top_.assign(n, 0);
}

StopChecker::StopChecker(uint32_t n, uint32_t mode, uint32_t k, double eps, uint64_t omega,
                         const double *L_l, const double *L_u, Groups &&groups)
    : n_(n), mode_(mode), k_(k), eps_(eps), omega_(omega), Ll_(L_l), Lu_(L_u) {
  group_ = std::move(groups.of);
  gL_l_ = std::move(groups.L_l);
  gL_u_ = std::move(groups.L_u);
  gmax_.resize(gL_l_.size());
  if (mode_ == 1) in_top_.assign(n, 0);
}

bool StopChecker::check_group_max(const uint64_t *gmax, uint64_t tau, double *worst) const {
  const double T = (double)tau, W = (double)omega_;
  bool stop = true;
  double w = 0.0;
  for (size_t g = 0; g < gL_l_.size(); ++g) {
    const double bt = (double)gmax[g] / T;
    const double f = bound_f(bt, gL_l_[g], W, T), gg = bound_g(bt, gL_u_[g], W, T);
    if (!(f <= eps_) || !(gg <= eps_)) {
      stop = false;
      if (!worst) return false;
    }
    w = std::max(w, std::max(f, gg) / eps_);
  }
  if (worst) *worst = w;
  return stop;
}

// gmax_[g], seen_[g]: the largest count in group g and whether g has a node, over the
// nodes (those not marked in in_top_ when skip_top).  Ranges of nodes run on the worker
// threads and their maxima are merged (the result does not depend on the order); many
// groups or few nodes take one pass.
void StopChecker::group_maxima(const uint64_t *count, bool skip_top) {
  const size_t G = gmax_.size();
  std::fill(gmax_.begin(), gmax_.end(), 0);
  seen_.assign(G, 0);
  if (G > 4096 || parallel_threads(n_) == 1) {
    for (uint32_t v = 0; v < n_; ++v) {
      if (skip_top && in_top_[v]) continue;
      const uint32_t g = group_[v];
      seen_[g] = 1;
      gmax_[g] = std::max(gmax_[g], count[v]);
    }
    return;
  }
  const unsigned nw = workers().size();
  pgmax_.resize(nw);
  pseen_.resize(nw);
  pused_.assign(nw, 0);
  parallel_ranges(n_, [&](uint32_t vb, uint32_t ve, unsigned w) {
    std::vector<uint64_t> &gm = pgmax_[w];
    std::vector<uint8_t> &sn = pseen_[w];
    gm.assign(G, 0);
    sn.assign(G, 0);
    pused_[w] = 1;
    for (uint32_t v = vb; v < ve; ++v) {
      if (skip_top && in_top_[v]) continue;
      const uint32_t g = group_[v];
      sn[g] = 1;
      gm[g] = std::max(gm[g], count[v]);
    }
  });
  for (unsigned w = 0; w < nw; ++w) {
    if (!pused_[w]) continue;
    for (size_t g = 0; g < G; ++g) {
      seen_[g] |= pseen_[w][g];
      gmax_[g] = std::max(gmax_[g], pgmax_[w][g]);
    }
  }
}

bool StopChecker::check(const uint64_t *count, uint64_t tau) {
  const double T = (double)tau, W = (double)omega_;
  std::vector<uint8_t> &seen = seen_;
  if (mode_ == 0) {
    group_maxima(count, false);
    for (size_t g = 0; g < gmax_.size(); ++g) {
      if (!seen[g]) continue;
      const double bt = (double)gmax_[g] / T;
      if (!(bound_f(bt, gL_l_[g], W, T) <= eps_) || !(bound_g(bt, gL_u_[g], W, T) <= eps_))
        return false;
    }
    return true;
  }
  // top-k (Algorithm 3): the k+1 largest by (count desc, id asc) are handled one by one;
  // for the rest only the per-group maximum can decide the second loop's condition.
  const uint32_t head = std::min(n_, k_ + 1);
  // Counts never decrease between checks, so the k+1 largest now all have a count of
  // at least the (k+1)-th largest of the previous check: select among those only.
  // (the candidates in id order: a counting pass and a writing pass over ranges of nodes)
  {
    const unsigned nw = workers().size();
    std::vector<uint32_t> at(nw + 1, 0);
    parallel_ranges(n_, [&](uint32_t vb, uint32_t ve, unsigned w) {
      uint32_t c = 0;
      for (uint32_t v = vb; v < ve; ++v) c += count[v] >= head_floor_;
      at[w + 1] = c;
    });
    for (unsigned w = 0; w < nw; ++w) at[w + 1] += at[w];
    order_.resize(at[nw]);
    parallel_ranges(n_, [&](uint32_t vb, uint32_t ve, unsigned w) {
      uint32_t o = at[w];
      for (uint32_t v = vb; v < ve; ++v)
        if (count[v] >= head_floor_) order_[o++] = v;
    });
  }
  if (order_.size() < head) {  // cannot happen for non-decreasing counts; select among all
    order_.resize(n_);
    for (uint32_t v = 0; v < n_; ++v) order_[v] = v;
  }
  auto cmp = [count](uint32_t a, uint32_t b) {
    return count[a] != count[b] ? count[a] > count[b] : a < b;
  };
  if (order_.size() > 65536 && order_.size() > 8ull * head) {
    // many candidates (the first check): the head largest of each range of them on the
    // worker threads, then of those -- the order is total, so the set is the same
    const uint32_t C = (uint32_t)order_.size();
    const unsigned nw = workers().size();
    std::vector<uint32_t> rb(nw, C), kept(nw, 0);
    parallel_ranges(C, [&](uint32_t b, uint32_t e, unsigned w) {
      rb[w] = b;
      kept[w] = std::min(head, e - b);
      if (e - b > head)
        std::nth_element(order_.begin() + b, order_.begin() + b + (head - 1),
                         order_.begin() + e, cmp);
    });
    uint32_t o = 0;
    for (unsigned w = 0; w < nw; ++w)
      for (uint32_t i = 0; i < kept[w]; ++i) order_[o++] = order_[rb[w] + i];
    order_.resize(o);
  }
  std::nth_element(order_.begin(), order_.begin() + (head - 1), order_.end(), cmp);
  std::sort(order_.begin(), order_.begin() + head, cmp);
  head_floor_ = count[order_[head - 1]];
  auto bt = [&](uint32_t v) { return (double)count[v] / T; };
  auto fv = [&](uint32_t v) { return bound_f(bt(v), Ll_[v], W, T); };
  auto gv = [&](uint32_t v) { return bound_g(bt(v), Lu_[v], W, T); };
  for (uint32_t i = 0; i < k_; ++i) {
    const uint32_t v = order_[i];
    if (fv(v) > eps_ || gv(v) > eps_) {
      if (i > 0 && bt(order_[i - 1]) - fv(order_[i - 1]) < bt(v) + gv(v)) return false;
      if (i + 1 < n_ && bt(v) - fv(v) < bt(order_[i + 1]) + gv(order_[i + 1])) return false;
    }
  }
  const uint32_t vk = order_[k_ - 1];
  const double kth_low = bt(vk) - fv(vk);
  for (uint32_t i = 0; i < k_; ++i) in_top_[order_[i]] = 1;
  group_maxima(count, true);
  for (uint32_t i = 0; i < k_; ++i) in_top_[order_[i]] = 0;
  for (size_t g = 0; g < gmax_.size(); ++g) {
    if (!seen[g]) continue;
    const double b = (double)gmax_[g] / T;
    const double f = bound_f(b, gL_l_[g], W, T), gg = bound_g(b, gL_u_[g], W, T);
    if ((f > eps_ || gg > eps_) && kth_low < b + gg) return false;
  }
  return true;
}

// ------------------------------------------------------------------ rank intervals

void rank_intervals(uint32_t n, const double *lower, const double *upper, uint32_t *rank_lo,
                    uint32_t *rank_hi) {
  std::vector<double> lo_sorted(lower, lower + n), up_sorted(upper, upper + n);
  std::sort(lo_sorted.begin(), lo_sorted.end());
  std::sort(up_sorted.begin(), up_sorted.end());
  for (uint32_t v = 0; v < n; ++v) {
    // #{w: lower(w) >= upper(v)}, minus v itself if it qualifies
    size_t ge = lo_sorted.end() - std::lower_bound(lo_sorted.begin(), lo_sorted.end(), upper[v]);
    if (lower[v] >= upper[v]) --ge;
    rank_lo[v] = (uint32_t)(1 + ge);
    // #{w: upper(w) > lower(v)}
    rank_hi[v] = (uint32_t)(up_sorted.end() -
                            std::upper_bound(up_sorted.begin(), up_sorted.end(), lower[v]));
  }
}

}  // namespace kad
