// Host-side statistics of the adaptive algorithm (library-internal interface).
// All binary64, compiled without FMA contraction.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <vector>

namespace kad {

// Run f(begin, end) over a static split of [0, n) on up to 16 threads (one thread for
// small n).  Used for per-node loops whose iterations are independent.
void parallel_ranges(uint32_t n, const std::function<void(uint32_t, uint32_t, unsigned)> &f);
unsigned parallel_threads(uint32_t n);
// Run f(0), ..., f(tasks - 1) on the same worker threads, one task per thread at a time.
void parallel_tasks(unsigned tasks, const std::function<void(unsigned)> &f);
unsigned worker_count();

uint64_t omega_of(double epsilon, double delta, uint32_t vd, double c);
uint64_t omega_edges_of(double epsilon, double delta, uint32_t vd, double c);
uint64_t alpha_of(uint64_t omega);
uint64_t interval_of(uint64_t omega);

double bound_f(double bt, double L, double omega, double tau);
double bound_g(double bt, double L, double omega, double tau);

// Returns 0 on success, -1 on invalid arguments.
int vertex_diameter(uint32_t n, uint64_t arcs, const uint32_t *row, const uint32_t *col,
                    const uint32_t *rrow, const uint32_t *rcol, double exact_limit, uint32_t *vd,
                    bool *exact);

// Node groups: nodes of one group have identical (L_l, L_u).
struct Groups {
  std::vector<uint32_t> of;    // node -> group
  std::vector<double> L_l, L_u; // group -> values
};

// computeDelta; optionally also returns a partition of the nodes into groups of
// identical (L_l, L_u) (not necessarily the coarsest one).
void compute_delta(uint32_t n, const uint64_t *count0, uint64_t alpha, uint64_t omega,
                   const double *lam_l, const double *lam_u, double delta, double eps_bal,
                   double *L_l, double *L_u, double *C, Groups *groups = nullptr);

// computeDelta for half-widths equal at every node, from the histogram of the pilot
// counts (hist[c] nodes have count c, c <= cmax): the arithmetic of compute_delta's
// uniform case, in its order.  Group g is the g-th count present in ascending order:
// cgrp[c] for every c with hist[c] > 0; groups.L_l/L_u per group; groups.of left empty.
void compute_delta_hist(uint32_t n, const uint64_t *hist, uint64_t cmax, uint64_t alpha,
                        uint64_t omega, double lam_l, double lam_u, double delta, double eps_bal,
                        std::vector<uint32_t> &cgrp, Groups &groups, double *C);

void topk_lambdas(uint32_t n, uint32_t k, const uint64_t *count0, uint64_t alpha, double eps,
                  double *lam_l, double *lam_u);

// The stopping check used inside a run.  Nodes sharing the same (L_l, L_u) pair are
// grouped once; f, g and b+g are non-decreasing in the count, so within a group only
// the largest count can decide a per-node condition.  Gives exactly the booleans of
// the plain evaluation.
class StopChecker {
 public:
  StopChecker(uint32_t n, uint32_t mode, uint32_t k, double eps, uint64_t omega,
              const double *L_l, const double *L_u);
  // with a known grouping (e.g. from compute_delta)
  StopChecker(uint32_t n, uint32_t mode, uint32_t k, double eps, uint64_t omega,
              const double *L_l, const double *L_u, Groups &&groups);
  // Counts passed to successive calls must not decrease (as within a run).
  bool check(const uint64_t *count, uint64_t tau);
  // All-nodes task only: the same decision from the per-group largest counts.  *worst
  // (optional) receives max over groups of max(f, g) / eps, how far the rule is from
  // stopping (a scheduling hint; the decision itself is f <= eps and g <= eps).
  bool check_group_max(const uint64_t *gmax, uint64_t tau, double *worst = nullptr) const;
  const std::vector<uint32_t> &group_of() const { return group_; }
  size_t groups() const { return gL_l_.size(); }

 private:
  uint32_t n_, mode_, k_;
  double eps_;
  uint64_t omega_;
  const double *Ll_, *Lu_;
  std::vector<uint32_t> group_;      // node -> group
  std::vector<double> gL_l_, gL_u_;  // group -> L values
  std::vector<uint64_t> gmax_;       // scratch: largest count per group
  std::vector<uint32_t> order_;      // scratch for the top-k order
  std::vector<uint8_t> in_top_, seen_;
  uint64_t head_floor_ = 0;          // (k+1)-th largest count at the last top-k check
  // per worker range: largest count and presence per group, and whether the range ran
  std::vector<std::vector<uint64_t>> pgmax_;
  std::vector<std::vector<uint8_t>> pseen_;
  std::vector<uint8_t> pused_;
  void group_maxima(const uint64_t *count, bool skip_top);
};

// Rank intervals of the top-k output: rank_lo = 1 + #{w != v: lower(w) >= upper(v)},
// rank_hi = #{w: upper(w) > lower(v)}.
void rank_intervals(uint32_t n, const double *lower, const double *upper, uint32_t *rank_lo,
                    uint32_t *rank_hi);

}  // namespace kad
