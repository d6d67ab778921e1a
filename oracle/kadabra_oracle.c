/*
 * KADABRA CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of what the sampled
 * betweenness hot path computes (Borassi & Natale, "KADABRA is an ADaptive
 * Algorithm for Betweenness via Random Approximation").  Only the test suite,
 * the smoke check and the bench's CPU-baseline leg may load it.  It shares no
 * code, headers or tables with the GPU library; the only thing the two have in
 * common is the written sampling procedure (the readings of the paper listed in
 * the design notes) and the seeded input graphs.
 *
 * Path counts are arbitrary-precision naturals (no 128-bit limit).  Floating
 * point is IEEE binary64, built with -ffp-contract=off; exp/log/sqrt are glibc.
 *
 * Parity status: every function below is pinned by a test against something
 * other than itself (numpy's Philox, Python integers, networkx shortest-path
 * counts and betweenness, closed forms, the paper's printed tables, exact
 * transition probabilities, the derivation's quadratic identities, arcs
 * scanned derived by hand from section 4's side rule on small gadgets, hand-
 * worked cases of Algorithm 3 and of section 5's half-widths).  The stopping
 * time tau of a whole run is pinned where it has a closed form (complete
 * graphs: every count is zero, so tau is the first check at which g(0) falls
 * to lambda) and elsewhere through Theorem 1's guarantee, tested over 200 seeds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ECAP (-3)      /* caller buffer too small */
#define OR_ERNG (-4)      /* rejection sampling exhausted its attempt budget */

#define UNSEEN 0xFFFFFFFFu
#define MAX_ATTEMPTS 64u  /* uniform_below gives up (error) after this many rejections */

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).                          */
/* A counter-based generator: 10 rounds of two 64x64->128 multiplications,     */
/* with the key bumped by two Weyl constants between rounds.                   */
/* ------------------------------------------------------------------------- */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream word 1 of the counter: (phase << 56) | (purpose << 48) | step. */
static uint64_t stream_word(uint32_t phase, uint32_t purpose, uint64_t step) {
  return ((uint64_t)phase << 56) | ((uint64_t)purpose << 48) | (step & 0xFFFFFFFFFFFFULL);
}

enum { PURPOSE_S = 0, PURPOSE_T = 1, PURPOSE_EDGE = 2, PURPOSE_BACK_S = 3, PURPOSE_BACK_T = 4 };

/* ------------------------------------------------------------------------- */
/* Arbitrary-precision natural numbers: little-endian 64-bit limbs.           */
/* The number of shortest paths can be exponential in the graph size (the    */
/* paper assumes O(1) arithmetic on them), so no fixed width is assumed here. */
/* ------------------------------------------------------------------------- */
typedef struct {
  uint32_t len; /* significant limbs; 0 encodes the value zero */
  uint32_t cap;
  uint64_t *d;
} nat;

static int nat_reserve(nat *a, uint32_t cap) {
  if (a->cap >= cap) return 0;
  uint32_t nc = a->cap ? a->cap : 2;
  while (nc < cap) nc *= 2;
  uint64_t *p = (uint64_t *)realloc(a->d, (size_t)nc * sizeof(uint64_t));
  if (!p) return -1;
  a->d = p;
  a->cap = nc;
  return 0;
}

static void nat_free(nat *a) {
  free(a->d);
  a->d = NULL;
  a->len = a->cap = 0;
}

static void nat_trim(nat *a) {
  while (a->len > 0 && a->d[a->len - 1] == 0) a->len--;
}

static int nat_set_u64(nat *a, uint64_t v) {
  if (v == 0) {
    a->len = 0;
    return 0;
  }
  if (nat_reserve(a, 1)) return -1;
  a->d[0] = v;
  a->len = 1;
  return 0;
}

static int nat_copy(nat *dst, const nat *src) {
  if (nat_reserve(dst, src->len ? src->len : 1)) return -1;
  if (src->len) memcpy(dst->d, src->d, (size_t)src->len * sizeof(uint64_t));
  dst->len = src->len;
  return 0;
}

/* acc += b */
static int nat_add(nat *acc, const nat *b) {
  uint32_t n = acc->len > b->len ? acc->len : b->len;
  if (nat_reserve(acc, n + 1)) return -1;
  for (uint32_t i = acc->len; i < n + 1; ++i) acc->d[i] = 0;
  uint64_t carry = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t bi = i < b->len ? b->d[i] : 0;
    unsigned __int128 s = (unsigned __int128)acc->d[i] + bi + carry;
    acc->d[i] = (uint64_t)s;
    carry = (uint64_t)(s >> 64);
  }
  acc->d[n] = carry;
  acc->len = n + 1;
  nat_trim(acc);
  return 0;
}

/* r = a * b (schoolbook); r must not alias a or b */
static int nat_mul(nat *r, const nat *a, const nat *b) {
  if (a->len == 0 || b->len == 0) {
    r->len = 0;
    return 0;
  }
  uint32_t n = a->len + b->len;
  if (nat_reserve(r, n)) return -1;
  memset(r->d, 0, (size_t)n * sizeof(uint64_t));
  for (uint32_t i = 0; i < a->len; ++i) {
    uint64_t carry = 0;
    for (uint32_t j = 0; j < b->len; ++j) {
      unsigned __int128 t = (unsigned __int128)a->d[i] * b->d[j] + r->d[i + j] + carry;
      r->d[i + j] = (uint64_t)t;
      carry = (uint64_t)(t >> 64);
    }
    r->d[i + b->len] = carry;
  }
  r->len = n;
  nat_trim(r);
  return 0;
}

static int nat_cmp(const nat *a, const nat *b) {
  if (a->len != b->len) return a->len < b->len ? -1 : 1;
  for (uint32_t i = a->len; i-- > 0;) {
    if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
  }
  return 0;
}

static int nat_is_one(const nat *a) { return a->len == 1 && a->d[0] == 1; }

/* number of significant bits */
static uint64_t nat_bitlen(const nat *a) {
  if (a->len == 0) return 0;
  uint64_t top = a->d[a->len - 1];
  return (uint64_t)(a->len - 1) * 64 + (64 - (uint64_t)__builtin_clzll(top));
}

/* a -= 1 (a > 0) */
static void nat_dec(nat *a) {
  for (uint32_t i = 0; i < a->len; ++i) {
    if (a->d[i]-- != 0) break;
  }
  nat_trim(a);
}

/* ------------------------------------------------------------------------- */
/* uniform_below(bound): an integer uniform in [0, bound).                     */
/* bound == 1 gives 0 and consumes nothing.  Otherwise W = bitlength(bound-1); */
/* attempt a takes ceil(W/64) words of the Philox stream                       */
/* (counter = (i, stream word, a, block)), least-significant word first, four  */
/* words per block, masks the result to W bits and accepts it if < bound.      */
/* ------------------------------------------------------------------------- */
static int uniform_below(const nat *bound, uint64_t seed, uint64_t i, uint64_t sword, nat *out,
                         nat *scratch) {
  if (nat_is_one(bound)) {
    out->len = 0;
    return OR_OK;
  }
  if (nat_copy(scratch, bound)) return OR_ENOMEM;
  nat_dec(scratch);
  uint64_t W = nat_bitlen(scratch);
  uint32_t q = (uint32_t)((W + 63) / 64);
  if (nat_reserve(out, q)) return OR_ENOMEM;
  const uint64_t key[2] = {seed, 0};
  for (uint32_t attempt = 0; attempt < MAX_ATTEMPTS; ++attempt) {
    uint64_t blk[4] = {0, 0, 0, 0};
    for (uint32_t j = 0; j < q; ++j) {
      if (j % 4 == 0) {
        const uint64_t ctr[4] = {i, sword, attempt, j / 4};
        or_philox4x64_10(ctr, key, blk);
      }
      out->d[j] = blk[j % 4];
    }
    uint32_t topbits = (uint32_t)(W - (uint64_t)(q - 1) * 64);
    if (topbits < 64) out->d[q - 1] &= (((uint64_t)1) << topbits) - 1;
    out->len = q;
    nat_trim(out);
    if (nat_cmp(out, bound) < 0) return OR_OK;
  }
  return OR_ERNG;
}

/* Exported for the pins: bound and out are little-endian 64-bit words. */
int or_uniform_below(const uint64_t *bound, uint32_t bound_words, uint64_t seed, uint64_t i,
                     uint32_t phase, uint32_t purpose, uint64_t step, uint64_t *out,
                     uint32_t out_words) {
  nat b = {0, 0, NULL}, r = {0, 0, NULL}, s = {0, 0, NULL};
  int rc = OR_OK;
  if (nat_reserve(&b, bound_words ? bound_words : 1)) return OR_ENOMEM;
  memcpy(b.d, bound, (size_t)bound_words * sizeof(uint64_t));
  b.len = bound_words;
  nat_trim(&b);
  if (b.len == 0) {
    rc = OR_EINVAL;
    goto done;
  }
  rc = uniform_below(&b, seed, i, stream_word(phase, purpose, step), &r, &s);
  if (rc == OR_OK) {
    if (r.len > out_words) {
      rc = OR_ECAP;
      goto done;
    }
    memset(out, 0, (size_t)out_words * sizeof(uint64_t));
    if (r.len) memcpy(out, r.d, (size_t)r.len * sizeof(uint64_t));
  }
done:
  nat_free(&b);
  nat_free(&r);
  nat_free(&s);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Graph: CSR out-rows, and in-rows (the transpose; identical when undirected) */
/* ------------------------------------------------------------------------- */
typedef struct {
  uint32_t n;
  uint64_t arcs;
  int32_t directed;
  const uint32_t *row, *col;   /* out-rows */
  const uint32_t *rrow, *rcol; /* in-rows */
} or_graph;

/* Per-thread working state of one sample. */
typedef struct {
  uint32_t n;
  uint32_t *dist_s, *dist_t; /* BFS level from s (forward) and from t (backward) */
  nat *sig_s, *sig_t;        /* number of shortest s->x and x->t paths */
  uint32_t *front_s, *front_t, *next;
  uint32_t *touched;
  size_t ntouched;
  uint32_t *sorted;
  nat tmp, tmp2, acc, r, bound, scratch;
} ows;

static void ows_free(ows *w) {
  if (!w) return;
  if (w->sig_s)
    for (uint32_t v = 0; v < w->n; ++v) nat_free(&w->sig_s[v]);
  if (w->sig_t)
    for (uint32_t v = 0; v < w->n; ++v) nat_free(&w->sig_t[v]);
  free(w->dist_s); free(w->dist_t); free(w->sig_s); free(w->sig_t);
  free(w->front_s); free(w->front_t); free(w->next); free(w->touched); free(w->sorted);
  nat_free(&w->tmp); nat_free(&w->tmp2); nat_free(&w->acc); nat_free(&w->r);
  nat_free(&w->bound); nat_free(&w->scratch);
  free(w);
}

static ows *ows_new(uint32_t n) {
  ows *w = (ows *)calloc(1, sizeof(ows));
  if (!w) return NULL;
  w->n = n;
  w->dist_s = (uint32_t *)malloc((size_t)n * 4);
  w->dist_t = (uint32_t *)malloc((size_t)n * 4);
  w->sig_s = (nat *)calloc(n, sizeof(nat));
  w->sig_t = (nat *)calloc(n, sizeof(nat));
  w->front_s = (uint32_t *)malloc((size_t)n * 4);
  w->front_t = (uint32_t *)malloc((size_t)n * 4);
  w->next = (uint32_t *)malloc((size_t)n * 4);
  w->touched = (uint32_t *)malloc((size_t)n * 2 * 4);
  w->sorted = (uint32_t *)malloc((size_t)n * 4);
  if (!w->dist_s || !w->dist_t || !w->sig_s || !w->sig_t || !w->front_s || !w->front_t ||
      !w->next || !w->touched || !w->sorted) {
    ows_free(w);
    return NULL;
  }
  for (uint32_t v = 0; v < n; ++v) w->dist_s[v] = w->dist_t[v] = UNSEEN;
  return w;
}

static void ows_reset(ows *w) {
  for (size_t k = 0; k < w->ntouched; ++k) {
    uint32_t v = w->touched[k];
    w->dist_s[v] = w->dist_t[v] = UNSEEN;
    w->sig_s[v].len = 0;
    w->sig_t[v].len = 0;
  }
  w->ntouched = 0;
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* One sample's outcome. */
typedef struct {
  uint32_t s, t;
  int32_t connected;   /* 0: s and t disconnected (no path, no hits) */
  uint32_t ls, lt;     /* levels of the two BFSs at the meeting */
  uint64_t arcs;       /* arcs scanned by level expansions */
  uint64_t sigma_bits; /* bit length of sigma_st (0 when disconnected) */
  uint32_t len;        /* number of path nodes, s..t inclusive */
  uint32_t *path;      /* caller-provided, room for n nodes */
} osample;

/*
 * One sample of the balanced bidirectional BFS (paper section 4, "Balanced
 * Bidirectional BFS"; pair drawing as in section 2, path uniform among the
 * shortest s-t paths).
 *
 *  - s uniform in [0,n), t uniform in [0,n) \ {s}.
 *  - Both sides keep a frontier (the nodes of their last level) and its degree
 *    sum; the side with the smaller sum is expanded (ties to the s side).  The
 *    s side follows out-arcs, the t side in-arcs.
 *  - Expanding a level: for every arc (u,w) out of the frontier, if w was
 *    reached from the other side the two searches touch; else if w is new it
 *    joins the next level with sigma(w) = sigma(u); else if w is in the next
 *    level sigma(w) += sigma(u) (Brandes' path counting).  The whole level is
 *    always finished.
 *  - Stop when the searches touched, or when the expanded side produced no new
 *    node (s and t disconnected: a sample with no hits).
 *  - At the meeting, the candidate edges are the arcs v->w with v on the s
 *    side's last level and w on the t side's last level; (v,w) is chosen with
 *    probability proportional to sigma_sv * sigma_wt, scanning v in increasing
 *    id and w in v's row order.  The two halves are completed by backtracking:
 *    a predecessor (s side, in-row order) or successor (t side, out-row order)
 *    on the level below, chosen with probability proportional to its count.
 *
 * With `forward` set the s side is always expanded: the plain BFS from s that
 * runs until the level reaching t is finished (the search of the samplers the
 * paper compares against in section 6, whose cost it calls m_avg).  The t side
 * keeps its level 0 = {t}, so the candidate edges are the arcs (v, t) out of
 * the s side's last level, and the path is uniform as well.
 */
static int sample_one(const or_graph *g, ows *w, uint64_t seed, uint32_t phase, uint64_t i,
                      int forward, osample *out) {
  int rc;
  const uint32_t n = g->n;
  /* pair */
  if (nat_set_u64(&w->bound, n)) return OR_ENOMEM;
  if ((rc = uniform_below(&w->bound, seed, i, stream_word(phase, PURPOSE_S, 0), &w->r,
                          &w->scratch)))
    return rc;
  uint32_t s = w->r.len ? (uint32_t)w->r.d[0] : 0;
  if (nat_set_u64(&w->bound, n - 1)) return OR_ENOMEM;
  if ((rc = uniform_below(&w->bound, seed, i, stream_word(phase, PURPOSE_T, 0), &w->r,
                          &w->scratch)))
    return rc;
  uint32_t tp = w->r.len ? (uint32_t)w->r.d[0] : 0;
  uint32_t t = tp + (tp >= s ? 1u : 0u);
  out->s = s;
  out->t = t;
  out->connected = 0;
  out->arcs = 0;
  out->sigma_bits = 0;
  out->len = 0;
  out->ls = out->lt = 0;

  /* initial levels */
  w->dist_s[s] = 0;
  nat_set_u64(&w->sig_s[s], 1);
  w->dist_t[t] = 0;
  nat_set_u64(&w->sig_t[t], 1);
  w->touched[w->ntouched++] = s;
  w->touched[w->ntouched++] = t;
  size_t nfs = 1, nft = 1;
  w->front_s[0] = s;
  w->front_t[0] = t;
  uint32_t ls = 0, lt = 0;
  uint64_t ds = (uint64_t)g->row[s + 1] - g->row[s];   /* out-degree sum of F_s */
  uint64_t dt = (uint64_t)g->rrow[t + 1] - g->rrow[t]; /* in-degree sum of F_t */
  int met = 0;

  for (;;) {
    int expand_s = forward || ds <= dt;
    const uint32_t *rp = expand_s ? g->row : g->rrow;
    const uint32_t *cl = expand_s ? g->col : g->rcol;
    uint32_t *dist_me = expand_s ? w->dist_s : w->dist_t;
    uint32_t *dist_other = expand_s ? w->dist_t : w->dist_s;
    nat *sig_me = expand_s ? w->sig_s : w->sig_t;
    uint32_t *front = expand_s ? w->front_s : w->front_t;
    size_t nf = expand_s ? nfs : nft;
    uint32_t lvl = expand_s ? ls : lt;
    size_t nn = 0;
    uint64_t dnext = 0;
    for (size_t k = 0; k < nf; ++k) {
      uint32_t u = front[k];
      for (uint32_t j = rp[u]; j < rp[u + 1]; ++j) {
        uint32_t x = cl[j];
        out->arcs++;
        if (dist_other[x] != UNSEEN) {
          met = 1;
        } else if (dist_me[x] == UNSEEN) {
          dist_me[x] = lvl + 1;
          if (nat_copy(&sig_me[x], &sig_me[u])) return OR_ENOMEM;
          w->next[nn++] = x;
          w->touched[w->ntouched++] = x;
          dnext += (uint64_t)rp[x + 1] - rp[x];
        } else if (dist_me[x] == lvl + 1) {
          if (nat_add(&sig_me[x], &sig_me[u])) return OR_ENOMEM;
        }
      }
    }
    if (met) break;
    if (nn == 0) { /* disconnected */
      ows_reset(w);
      return OR_OK;
    }
    memcpy(front, w->next, nn * sizeof(uint32_t));
    if (expand_s) {
      nfs = nn;
      ls++;
      ds = dnext;
    } else {
      nft = nn;
      lt++;
      dt = dnext;
    }
  }

  /* candidate edges in canonical order: v ascending, then v's out-row order */
  memcpy(w->sorted, w->front_s, nfs * sizeof(uint32_t));
  qsort(w->sorted, nfs, sizeof(uint32_t), cmp_u32);
  nat *total = &w->acc;
  total->len = 0;
  for (size_t k = 0; k < nfs; ++k) {
    uint32_t v = w->sorted[k];
    for (uint32_t j = g->row[v]; j < g->row[v + 1]; ++j) {
      uint32_t x = g->col[j];
      if (w->dist_t[x] == lt) {
        if (nat_mul(&w->tmp, &w->sig_s[v], &w->sig_t[x])) return OR_ENOMEM;
        if (nat_add(total, &w->tmp)) return OR_ENOMEM;
      }
    }
  }
  out->sigma_bits = nat_bitlen(total);
  if ((rc = uniform_below(total, seed, i, stream_word(phase, PURPOSE_EDGE, 0), &w->r,
                          &w->scratch)))
    return rc;
  uint32_t mv = UNSEEN, mw = UNSEEN;
  w->tmp2.len = 0; /* prefix sum */
  for (size_t k = 0; k < nfs && mv == UNSEEN; ++k) {
    uint32_t v = w->sorted[k];
    for (uint32_t j = g->row[v]; j < g->row[v + 1]; ++j) {
      uint32_t x = g->col[j];
      if (w->dist_t[x] == lt) {
        if (nat_mul(&w->tmp, &w->sig_s[v], &w->sig_t[x])) return OR_ENOMEM;
        if (nat_add(&w->tmp2, &w->tmp)) return OR_ENOMEM;
        if (nat_cmp(&w->tmp2, &w->r) > 0) {
          mv = v;
          mw = x;
          break;
        }
      }
    }
  }
  if (mv == UNSEEN) return OR_EINVAL; /* cannot happen: r < total */

  /* s half: from v down to s, predecessors with probability prop. to sigma_s */
  uint32_t len = ls + lt + 2;
  out->path[ls] = mv;
  uint32_t x = mv;
  for (uint32_t j = ls; j >= 1; --j) {
    if ((rc = uniform_below(&w->sig_s[x], seed, i, stream_word(phase, PURPOSE_BACK_S, j), &w->r,
                            &w->scratch)))
      return rc;
    w->tmp2.len = 0;
    uint32_t pick = UNSEEN;
    for (uint32_t k = g->rrow[x]; k < g->rrow[x + 1]; ++k) {
      uint32_t u = g->rcol[k];
      if (w->dist_s[u] == j - 1) {
        if (nat_add(&w->tmp2, &w->sig_s[u])) return OR_ENOMEM;
        if (nat_cmp(&w->tmp2, &w->r) > 0) {
          pick = u;
          break;
        }
      }
    }
    if (pick == UNSEEN) return OR_EINVAL;
    x = pick;
    out->path[j - 1] = x;
  }
  /* t half: from w up to t, successors with probability prop. to sigma_t */
  uint32_t y = mw;
  out->path[ls + 1] = y;
  for (uint32_t j = lt; j >= 1; --j) {
    if ((rc = uniform_below(&w->sig_t[y], seed, i, stream_word(phase, PURPOSE_BACK_T, j), &w->r,
                            &w->scratch)))
      return rc;
    w->tmp2.len = 0;
    uint32_t pick = UNSEEN;
    for (uint32_t k = g->row[y]; k < g->row[y + 1]; ++k) {
      uint32_t z = g->col[k];
      if (w->dist_t[z] == j - 1) {
        if (nat_add(&w->tmp2, &w->sig_t[z])) return OR_ENOMEM;
        if (nat_cmp(&w->tmp2, &w->r) > 0) {
          pick = z;
          break;
        }
      }
    }
    if (pick == UNSEEN) return OR_EINVAL;
    y = pick;
    out->path[ls + 1 + (lt - j) + 1] = y;
  }
  out->connected = 1;
  out->ls = ls;
  out->lt = lt;
  out->len = len;
  ows_reset(w);
  return OR_OK;
}

/*
 * Samples with ids [first, first+count) of one phase.  Per sample: s, t, the
 * path (s..t, empty when disconnected) packed at path_nodes[path_off[k] ..
 * path_off[k+1]), the arcs scanned and the bit length of sigma_st.  Samples
 * are independent, so the threads only split the id range.
 */
int or_sample_paths_search(const or_graph *g, uint64_t seed, uint32_t phase, uint64_t first,
                           uint64_t count, int threads, int forward, uint32_t *s_out,
                           uint32_t *t_out, uint64_t *path_off, uint32_t *path_nodes,
                           uint64_t path_cap, uint64_t *arcs_out, uint64_t *sigma_bits_out) {
  if (!g || g->n < 2) return OR_EINVAL;
  uint32_t *lens = (uint32_t *)calloc(count ? count : 1, sizeof(uint32_t));
  uint32_t **paths = (uint32_t **)calloc(count ? count : 1, sizeof(uint32_t *));
  if (!lens || !paths) {
    free(lens);
    free(paths);
    return OR_ENOMEM;
  }
  int err = OR_OK;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
#pragma omp parallel
  {
    ows *w = ows_new(g->n);
    uint32_t *buf = (uint32_t *)malloc((size_t)g->n * sizeof(uint32_t));
    if (!w || !buf) {
#pragma omp critical
      err = OR_ENOMEM;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t k = 0; k < (int64_t)count; ++k) {
      if (err || !w || !buf) continue;
      osample o;
      o.path = buf;
      int rc = sample_one(g, w, seed, phase, first + (uint64_t)k, forward, &o);
      if (rc) {
#pragma omp critical
        err = rc;
        continue;
      }
      if (s_out) s_out[k] = o.s;
      if (t_out) t_out[k] = o.t;
      if (arcs_out) arcs_out[k] = o.arcs;
      if (sigma_bits_out) sigma_bits_out[k] = o.sigma_bits;
      lens[k] = o.len;
      if (o.len) {
        paths[k] = (uint32_t *)malloc((size_t)o.len * sizeof(uint32_t));
        if (!paths[k]) {
#pragma omp critical
          err = OR_ENOMEM;
          continue;
        }
        memcpy(paths[k], buf, (size_t)o.len * sizeof(uint32_t));
      }
    }
    ows_free(w);
    free(buf);
  }
  if (!err && path_off) {
    uint64_t off = 0;
    for (uint64_t k = 0; k < count; ++k) {
      path_off[k] = off;
      if (off + lens[k] > path_cap) {
        err = OR_ECAP;
        break;
      }
      if (lens[k]) memcpy(path_nodes + off, paths[k], (size_t)lens[k] * sizeof(uint32_t));
      off += lens[k];
    }
    if (!err) path_off[count] = off;
  }
  for (uint64_t k = 0; k < count; ++k) free(paths[k]);
  free(paths);
  free(lens);
  return err;
}

/* The balanced bidirectional search (section 4). */
int or_sample_paths(const or_graph *g, uint64_t seed, uint32_t phase, uint64_t first,
                    uint64_t count, int threads, uint32_t *s_out, uint32_t *t_out,
                    uint64_t *path_off, uint32_t *path_nodes, uint64_t path_cap,
                    uint64_t *arcs_out, uint64_t *sigma_bits_out) {
  return or_sample_paths_search(g, seed, phase, first, count, threads, 0, s_out, t_out,
                                path_off, path_nodes, path_cap, arcs_out, sigma_bits_out);
}

/* Hits of samples [first, first+count): count[v] += 1 for every interior node
 * v of each sampled path (section 2: X_i(v) = 1 iff v is on the path and
 * differs from s and t).  Adds the arcs scanned to *arcs. */
static int add_hits(const or_graph *g, uint64_t seed, uint32_t phase, uint64_t first,
                    uint64_t count, int threads, int forward, uint64_t *cnt, uint64_t *arcs) {
  if (count == 0) return OR_OK;
  uint64_t cap = count * (uint64_t)(g->n < 64 ? g->n : 64) + 1;
  uint64_t *off = (uint64_t *)malloc((count + 1) * sizeof(uint64_t));
  uint64_t *ar = (uint64_t *)malloc(count * sizeof(uint64_t));
  uint32_t *nodes = NULL;
  int rc;
  for (;;) {
    nodes = (uint32_t *)malloc(cap * sizeof(uint32_t));
    if (!off || !ar || !nodes) {
      rc = OR_ENOMEM;
      break;
    }
    rc = or_sample_paths_search(g, seed, phase, first, count, threads, forward, NULL, NULL, off,
                                nodes, cap, ar, NULL);
    if (rc != OR_ECAP) break;
    free(nodes);
    nodes = NULL;
    cap *= 4;
  }
  if (rc == OR_OK) {
    for (uint64_t k = 0; k < count; ++k) {
      *arcs += ar[k];
      uint64_t a = off[k], b = off[k + 1];
      for (uint64_t j = a + 1; j + 1 < b; ++j) cnt[nodes[j]] += 1;
    }
  }
  free(off);
  free(ar);
  free(nodes);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Edge betweenness (section 1: the method adapts to the centrality of edges):  */
/* bc(e) = 1/(n(n-1)) * sum over ordered pairs s != t of sigma_st(e)/sigma_st,   */
/* with sigma_st(e) the shortest s-t paths through e; a sample hits every edge  */
/* of its path.  Edge ids: a directed graph's edge is its arc's CSR position; an */
/* undirected edge {u, v} is the rank of its arc u -> v (u < v) in CSR order,    */
/* and both of its arcs map to that id.                                         */
/* ------------------------------------------------------------------------- */
uint64_t or_edge_count(const or_graph *g) { return g->directed ? g->arcs : g->arcs / 2; }

/* position of the arc a -> b in a's out-row (rows are sorted), or UINT64_MAX */
static uint64_t arc_pos(const or_graph *g, uint32_t a, uint32_t b) {
  uint64_t lo = g->row[a], hi = g->row[a + 1];
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if (g->col[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  return (lo < g->row[a + 1] && g->col[lo] == b) ? lo : UINT64_MAX;
}

int or_edge_ids(const or_graph *g, uint32_t *eid) {
  if (g->directed) {
    for (uint64_t e = 0; e < g->arcs; ++e) eid[e] = (uint32_t)e;
    return OR_OK;
  }
  uint32_t next = 0;
  for (uint32_t u = 0; u < g->n; ++u) {
    for (uint32_t e = g->row[u]; e < g->row[u + 1]; ++e) {
      uint32_t v = g->col[e];
      if (v < u) continue;
      uint64_t back = arc_pos(g, v, u);
      if (back == UINT64_MAX) return OR_EINVAL; /* not symmetric */
      eid[e] = next;
      eid[back] = next;
      next++;
    }
  }
  return OR_OK;
}

/* hits of samples [first, first+count) on the edges of their paths: cnt[eid] += 1 */
static int add_edge_hits(const or_graph *g, uint64_t seed, uint32_t phase, uint64_t first,
                         uint64_t count, int threads, int forward, const uint32_t *eid,
                         uint64_t *cnt, uint64_t *arcs) {
  if (count == 0) return OR_OK;
  uint64_t cap = count * (uint64_t)(g->n < 64 ? g->n : 64) + 1;
  uint64_t *off = (uint64_t *)malloc((count + 1) * sizeof(uint64_t));
  uint64_t *ar = (uint64_t *)malloc(count * sizeof(uint64_t));
  uint32_t *nodes = NULL;
  int rc;
  for (;;) {
    nodes = (uint32_t *)malloc(cap * sizeof(uint32_t));
    if (!off || !ar || !nodes) {
      rc = OR_ENOMEM;
      break;
    }
    rc = or_sample_paths_search(g, seed, phase, first, count, threads, forward, NULL, NULL, off,
                                nodes, cap, ar, NULL);
    if (rc != OR_ECAP) break;
    free(nodes);
    nodes = NULL;
    cap *= 4;
  }
  if (rc == OR_OK) {
    for (uint64_t k = 0; k < count && rc == OR_OK; ++k) {
      *arcs += ar[k];
      for (uint64_t j = off[k]; j + 1 < off[k + 1]; ++j) {
        uint64_t pos = arc_pos(g, nodes[j], nodes[j + 1]);
        if (pos == UINT64_MAX) {
          rc = OR_EINVAL; /* cannot happen: consecutive path nodes are adjacent */
          break;
        }
        cnt[eid[pos]] += 1;
      }
    }
  }
  free(off);
  free(ar);
  free(nodes);
  return rc;
}

int or_edge_hits(const or_graph *g, uint64_t seed, uint32_t phase, uint64_t first,
                 uint64_t count, int threads, int forward, uint64_t *cnt, uint64_t *arcs) {
  uint32_t *eid = (uint32_t *)malloc((g->arcs ? g->arcs : 1) * sizeof(uint32_t));
  if (!eid) return OR_ENOMEM;
  int rc = or_edge_ids(g, eid);
  uint64_t a = 0;
  if (rc == OR_OK) rc = add_edge_hits(g, seed, phase, first, count, threads, forward, eid, cnt, &a);
  if (arcs) *arcs = a;
  free(eid);
  return rc;
}

/* Exact edge betweenness by Brandes' dependencies: from each source s, an edge (v, w) of the
 * shortest-path DAG carries sigma_sv / sigma_sw * (1 + delta_s(w)) of the pairs (s, t). */
int or_edge_brandes(const or_graph *g, double *ebc) {
  uint32_t n = g->n;
  uint64_t me = or_edge_count(g);
  uint32_t *eid = (uint32_t *)malloc((g->arcs ? g->arcs : 1) * 4);
  uint32_t *dist = (uint32_t *)malloc((size_t)n * 4);
  uint32_t *order = (uint32_t *)malloc((size_t)n * 4);
  double *sig = (double *)malloc((size_t)n * 8);
  double *dep = (double *)malloc((size_t)n * 8);
  if (!eid || !dist || !order || !sig || !dep) {
    free(eid); free(dist); free(order); free(sig); free(dep);
    return OR_ENOMEM;
  }
  int rc = or_edge_ids(g, eid);
  for (uint64_t e = 0; e < me; ++e) ebc[e] = 0.0;
  for (uint32_t s = 0; s < n && rc == OR_OK; ++s) {
    for (uint32_t v = 0; v < n; ++v) {
      dist[v] = UNSEEN;
      sig[v] = 0.0;
      dep[v] = 0.0;
    }
    size_t head = 0, tail = 0;
    dist[s] = 0;
    sig[s] = 1.0;
    order[tail++] = s;
    while (head < tail) {
      uint32_t u = order[head++];
      for (uint32_t j = g->row[u]; j < g->row[u + 1]; ++j) {
        uint32_t x = g->col[j];
        if (dist[x] == UNSEEN) {
          dist[x] = dist[u] + 1;
          order[tail++] = x;
        }
        if (dist[x] == dist[u] + 1) sig[x] += sig[u];
      }
    }
    for (size_t k = tail; k-- > 0;) {
      uint32_t u = order[k];
      for (uint32_t j = g->row[u]; j < g->row[u + 1]; ++j) {
        uint32_t x = g->col[j];
        if (dist[x] == dist[u] + 1) {
          double c = sig[u] / sig[x] * (1.0 + dep[x]);
          ebc[eid[j]] += c;
          dep[u] += c;
        }
      }
    }
  }
  double norm = 1.0 / ((double)n * (double)(n - 1));
  for (uint64_t e = 0; e < me; ++e) ebc[e] *= norm;
  free(eid); free(dist); free(order); free(sig); free(dep);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Vertex diameter VD: the largest number of nodes on a shortest path.         */
/* Exact (a BFS from every node) when n * arcs <= 1e9; otherwise an upper      */
/* bound: a shortest path crosses strongly connected components along a path  */
/* of the condensation DAG and, inside a component C, is a shortest path of    */
/* G[C], so it has at most ecc_out_C(r) + ecc_in_C(r) + 1 nodes for any r in C  */
/* (r = the node of C with the largest in+out degree, lowest id on ties).  The */
/* bound is the heaviest DAG path under those component weights.              */
/* ------------------------------------------------------------------------- */
static uint32_t bfs_ecc(uint32_t n, const uint32_t *rp, const uint32_t *cl, uint32_t src,
                        const uint32_t *comp, uint32_t restrict_comp, uint32_t *dist,
                        uint32_t *queue) {
  size_t head = 0, tail = 0;
  dist[src] = 0;
  queue[tail++] = src;
  uint32_t ecc = 0;
  while (head < tail) {
    uint32_t u = queue[head++];
    if (dist[u] > ecc) ecc = dist[u];
    for (uint32_t j = rp[u]; j < rp[u + 1]; ++j) {
      uint32_t x = cl[j];
      if (comp && comp[x] != restrict_comp) continue;
      if (dist[x] == UNSEEN) {
        dist[x] = dist[u] + 1;
        queue[tail++] = x;
      }
    }
  }
  for (size_t k = 0; k < tail; ++k) dist[queue[k]] = UNSEEN;
  (void)n;
  return ecc;
}

/* Strongly connected components by Kosaraju's two passes (iterative DFS).
 * comp[v] in [0, ncomp); components are numbered in a topological order of
 * the condensation (every arc goes from a lower to a higher or equal id). */
static int scc(const or_graph *g, uint32_t *comp, uint32_t *ncomp) {
  uint32_t n = g->n;
  uint32_t *order = (uint32_t *)malloc((size_t)n * 4);
  uint32_t *stack = (uint32_t *)malloc((size_t)n * 4);
  uint32_t *it = (uint32_t *)malloc((size_t)n * 4);
  uint8_t *seen = (uint8_t *)calloc(n, 1);
  if (!order || !stack || !it || !seen) {
    free(order); free(stack); free(it); free(seen);
    return OR_ENOMEM;
  }
  size_t no = 0;
  /* pass 1: finishing order on out-arcs */
  for (uint32_t r = 0; r < n; ++r) {
    if (seen[r]) continue;
    size_t sp = 0;
    stack[sp++] = r;
    seen[r] = 1;
    it[r] = g->row[r];
    while (sp) {
      uint32_t u = stack[sp - 1];
      if (it[u] < g->row[u + 1]) {
        uint32_t x = g->col[it[u]++];
        if (!seen[x]) {
          seen[x] = 1;
          it[x] = g->row[x];
          stack[sp++] = x;
        }
      } else {
        order[no++] = u;
        sp--;
      }
    }
  }
  /* pass 2: in-arcs, in reverse finishing order */
  for (uint32_t v = 0; v < n; ++v) comp[v] = UNSEEN;
  uint32_t c = 0;
  for (size_t k = n; k-- > 0;) {
    uint32_t r = order[k];
    if (comp[r] != UNSEEN) continue;
    size_t sp = 0;
    stack[sp++] = r;
    comp[r] = c;
    while (sp) {
      uint32_t u = stack[--sp];
      for (uint32_t j = g->rrow[u]; j < g->rrow[u + 1]; ++j) {
        uint32_t x = g->rcol[j];
        if (comp[x] == UNSEEN) {
          comp[x] = c;
          stack[sp++] = x;
        }
      }
    }
    c++;
  }
  *ncomp = c;
  free(order); free(stack); free(it); free(seen);
  return OR_OK;
}

int or_vertex_diameter(const or_graph *g, double exact_limit, uint32_t *vd, int32_t *exact) {
  uint32_t n = g->n;
  uint32_t *dist = (uint32_t *)malloc((size_t)n * 4);
  uint32_t *queue = (uint32_t *)malloc((size_t)n * 4);
  if (!dist || !queue) {
    free(dist); free(queue);
    return OR_ENOMEM;
  }
  for (uint32_t v = 0; v < n; ++v) dist[v] = UNSEEN;
  int rc = OR_OK;
  if ((double)n * (double)g->arcs <= exact_limit) {
    uint32_t best = 0;
    for (uint32_t v = 0; v < n; ++v) {
      uint32_t e = bfs_ecc(n, g->row, g->col, v, NULL, 0, dist, queue);
      if (e > best) best = e;
    }
    *vd = best + 1;
    *exact = 1;
  } else {
    uint32_t *comp = (uint32_t *)malloc((size_t)n * 4);
    uint32_t nc = 0;
    if (!comp || (rc = scc(g, comp, &nc))) {
      free(comp); free(dist); free(queue);
      return rc ? rc : OR_ENOMEM;
    }
    uint32_t *root = (uint32_t *)malloc((size_t)nc * 4);
    uint64_t *rdeg = (uint64_t *)calloc(nc, 8);
    uint64_t *best = (uint64_t *)calloc(nc, 8);
    if (!root || !rdeg || !best) {
      free(comp); free(dist); free(queue); free(root); free(rdeg); free(best);
      return OR_ENOMEM;
    }
    for (uint32_t c = 0; c < nc; ++c) root[c] = UNSEEN;
    for (uint32_t v = 0; v < n; ++v) {
      uint64_t d = (uint64_t)(g->row[v + 1] - g->row[v]) + (g->rrow[v + 1] - g->rrow[v]);
      uint32_t c = comp[v];
      if (root[c] == UNSEEN || d > rdeg[c]) {
        root[c] = v;
        rdeg[c] = d;
      }
    }
    /* component weights, then heaviest path over the DAG in topological order */
    uint64_t answer = 0;
    uint32_t *members_off = (uint32_t *)calloc((size_t)nc + 1, 4);
    uint32_t *members = (uint32_t *)malloc((size_t)n * 4);
    for (uint32_t v = 0; v < n; ++v) members_off[comp[v] + 1]++;
    for (uint32_t c = 0; c < nc; ++c) members_off[c + 1] += members_off[c];
    uint32_t *fill = (uint32_t *)malloc((size_t)nc * 4);
    memcpy(fill, members_off, (size_t)nc * 4);
    for (uint32_t v = 0; v < n; ++v) members[fill[comp[v]]++] = v;
    for (uint32_t c = 0; c < nc; ++c) {
      uint32_t r = root[c];
      uint64_t w = (uint64_t)bfs_ecc(n, g->row, g->col, r, comp, c, dist, queue) +
                   bfs_ecc(n, g->rrow, g->rcol, r, comp, c, dist, queue) + 1;
      /* best path ending in c: weight of c plus the best over predecessors;
       * predecessors have lower component ids and are already final */
      uint64_t pred = 0;
      for (uint32_t k = members_off[c]; k < members_off[c + 1]; ++k) {
        uint32_t v = members[k];
        for (uint32_t j = g->rrow[v]; j < g->rrow[v + 1]; ++j) {
          uint32_t c2 = comp[g->rcol[j]];
          if (c2 != c && best[c2] > pred) pred = best[c2];
        }
      }
      best[c] = pred + w;
      if (best[c] > answer) answer = best[c];
    }
    *vd = (uint32_t)(answer > 0xFFFFFFFFu ? 0xFFFFFFFFu : answer);
    *exact = 0;
    free(comp); free(root); free(rdeg); free(best); free(members_off); free(members); free(fill);
  }
  free(dist);
  free(queue);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Sample budget (Algorithm 1, first line): omega = c / lambda^2 *             */
/* (floor(log2(VD - 2)) + 1 + ln(2 / delta)), rounded up; floor(log2(x)) is    */
/* taken as 0 for VD <= 3.                                                     */
/* ------------------------------------------------------------------------- */
static uint32_t floor_log2_u32(uint32_t x) {
  uint32_t r = 0;
  while (x >= 2) {
    x >>= 1;
    r++;
  }
  return r;
}

uint64_t or_omega(double lambda, double delta, uint32_t vd, double c) {
  uint32_t base = vd > 3 ? vd - 2 : 1;
  double j = (double)(floor_log2_u32(base) + 1);
  double x = c / (lambda * lambda) * (j + log(2.0 / delta));
  return (uint64_t)ceil(x);
}

/* The same cap for edge betweenness: a shortest path has at most VD - 1 edges, so the
 * ranges "paths through edge e" shatter at most floor(log2(VD - 1)) + 1 paths (a path in
 * a shattered set of k lies in 2^(k-1) distinct ranges, each one of its edges), where the
 * node ranges give floor(log2(VD - 2)) + 1. */
uint64_t or_omega_edges(double lambda, double delta, uint32_t vd, double c) {
  uint32_t base = vd > 2 ? vd - 1 : 1;
  double j = (double)(floor_log2_u32(base) + 1);
  double x = c / (lambda * lambda) * (j + log(2.0 / delta));
  return (uint64_t)ceil(x);
}

/* Pilot size alpha = omega / 100 (Algorithm 2), at least one sample. */
uint64_t or_alpha(uint64_t omega) {
  uint64_t a = omega / 100;
  return a ? a : 1;
}

/* Default check interval: 2^floor(log2(omega/16)) clamped to [1024, 65536]. */
uint64_t or_default_interval(uint64_t omega) {
  uint64_t x = omega / 16;
  uint64_t b = 1;
  while (b * 2 <= x) b *= 2;
  if (b < 1024) b = 1024;
  if (b > 65536) b = 65536;
  return b;
}

/* ------------------------------------------------------------------------- */
/* f and g of Theorem azuma-borassi (appendix "Proof of Theorem 1"), with      */
/* L = log(1/delta_L) (resp. log(1/delta_U)) and bt = count / tau.            */
/* f is evaluated after multiplying by the conjugate, which is the same value */
/* in exact arithmetic but avoids the cancellation of (1/3 - omega/tau) + sqrt */
/* (the first term is negative because tau <= omega).                         */
/* ------------------------------------------------------------------------- */
double or_f(double bt, double L, double omega, double tau) {
  double a = 1.0 / 3.0 - omega / tau;
  double x = 2.0 * bt * omega / L;
  return (L / tau) * (x / (sqrt(a * a + x) - a));
}

double or_g(double bt, double L, double omega, double tau) {
  double b = 1.0 / 3.0 + omega / tau;
  double x = 2.0 * bt * omega / L;
  return (L / tau) * (b + sqrt(b * b + x));
}

/* ------------------------------------------------------------------------- */
/* computeDelta (Algorithm 2; appendix "How to choose delta_L, delta_U").      */
/* From the pilot estimate b0(v) = count0(v)/alpha and the wanted half-widths */
/* lambda_L(v), lambda_U(v): c_L = 2 b0 omega / lambda_L^2 (same for U); the   */
/* smallest C with S(C) = sum exp(-C/c) <= delta/2 - eps*delta is found by      */
/* bisection, and delta_L(v) = exp(-C/c_L(v)) + eps*delta/(2n).  Returned as   */
/* L_L = -ln(delta_L), L_U = -ln(delta_U).                                     */
/* S(C) is summed as sum_j mult_j * exp(-C/c_j) over the distinct values c_j  */
/* of the 2n constants in increasing order (exp(-C/0) taken as 0).             */
/* ------------------------------------------------------------------------- */
static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static double e_term(double C, double c) { return c == 0.0 ? 0.0 : exp(-C / c); }

static double s_of_c(double C, const double *vals, const uint64_t *mult, size_t nd) {
  double s = 0.0;
  for (size_t j = 0; j < nd; ++j) s += (double)mult[j] * e_term(C, vals[j]);
  return s;
}

int or_compute_delta(uint32_t n, const uint64_t *count0, uint64_t alpha, uint64_t omega,
                     const double *lam_l, const double *lam_u, double delta, double eps_bal,
                     double *L_l, double *L_u, double *C_out) {
  double *cl = (double *)malloc((size_t)n * sizeof(double));
  double *cu = (double *)malloc((size_t)n * sizeof(double));
  double *all = (double *)malloc((size_t)n * 2 * sizeof(double));
  uint64_t *mult = (uint64_t *)malloc((size_t)n * 2 * sizeof(uint64_t));
  if (!cl || !cu || !all || !mult) {
    free(cl); free(cu); free(all); free(mult);
    return OR_ENOMEM;
  }
  for (uint32_t v = 0; v < n; ++v) {
    double b0 = (double)count0[v] / (double)alpha;
    cl[v] = 2.0 * b0 * (double)omega / (lam_l[v] * lam_l[v]);
    cu[v] = 2.0 * b0 * (double)omega / (lam_u[v] * lam_u[v]);
    all[2 * (size_t)v] = cl[v];
    all[2 * (size_t)v + 1] = cu[v];
  }
  qsort(all, (size_t)n * 2, sizeof(double), cmp_double);
  size_t nd = 0;
  for (size_t k = 0; k < (size_t)n * 2; ++k) {
    if (nd > 0 && all[nd - 1] == all[k]) {
      mult[nd - 1]++;
    } else {
      all[nd] = all[k];
      mult[nd] = 1;
      nd++;
    }
  }
  double target = delta / 2.0 - eps_bal * delta;
  double lo = 0.0, hi = 1.0;
  while (s_of_c(hi, all, mult, nd) > target) hi *= 2.0;
  for (int it = 0; it < 100; ++it) {
    double mid = (lo + hi) / 2.0;
    if (s_of_c(mid, all, mult, nd) > target)
      lo = mid;
    else
      hi = mid;
  }
  double C = hi;
  double add = eps_bal * delta / (2.0 * (double)n);
  for (uint32_t v = 0; v < n; ++v) {
    L_l[v] = -log(e_term(C, cl[v]) + add);
    L_u[v] = -log(e_term(C, cu[v]) + add);
  }
  if (C_out) *C_out = C;
  free(cl); free(cu); free(all); free(mult);
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Stopping conditions                                                         */
/* ------------------------------------------------------------------------- */

/* All centralities within lambda (section 2): stop when f <= lambda and
 * g <= lambda at every node. */
int or_stop_all(uint32_t n, const uint64_t *count, uint64_t tau, uint64_t omega, double lambda,
                const double *L_l, const double *L_u) {
  double T = (double)tau, W = (double)omega;
  for (uint32_t v = 0; v < n; ++v) {
    double bt = (double)count[v] / T;
    if (!(or_f(bt, L_l[v], W, T) <= lambda)) return 0;
    if (!(or_g(bt, L_u[v], W, T) <= lambda)) return 0;
  }
  return 1;
}

/* order: count descending, id ascending */
static const uint64_t *g_sort_count;
static int cmp_rank(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  uint64_t cx = g_sort_count[x], cy = g_sort_count[y];
  if (cx != cy) return cx > cy ? -1 : 1;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static void rank_order(uint32_t n, const uint64_t *count, uint32_t *order) {
  for (uint32_t v = 0; v < n; ++v) order[v] = v;
  g_sort_count = count;
  qsort(order, n, sizeof(uint32_t), cmp_rank);
}

/* Top-k stopping condition (Algorithm 3), on the order v_1..v_n by estimate.
 * A position without a neighbour (v_0, v_{n+1}) is never "not separated". */
int or_stop_topk(uint32_t n, uint32_t k, const uint64_t *count, uint64_t tau, uint64_t omega,
                 double lambda, const double *L_l, const double *L_u) {
  uint32_t *ord = (uint32_t *)malloc((size_t)n * 4);
  if (!ord) return OR_ENOMEM;
  rank_order(n, count, ord);
  double T = (double)tau, W = (double)omega;
#define BT(v) ((double)count[v] / T)
#define FV(v) or_f(BT(v), L_l[v], W, T)
#define GV(v) or_g(BT(v), L_u[v], W, T)
  int stop = 1;
  for (uint32_t i = 0; i < k && stop; ++i) { /* positions 1..k */
    uint32_t v = ord[i];
    if (FV(v) > lambda || GV(v) > lambda) {
      int bad = 0;
      if (i > 0) {
        uint32_t p = ord[i - 1];
        if (BT(p) - FV(p) < BT(v) + GV(v)) bad = 1;
      }
      if (i + 1 < n) {
        uint32_t q = ord[i + 1];
        if (BT(v) - FV(v) < BT(q) + GV(q)) bad = 1;
      }
      if (bad) stop = 0;
    }
  }
  if (stop) {
    uint32_t vk = ord[k - 1];
    double lowk = BT(vk) - FV(vk);
    for (uint32_t i = k; i < n; ++i) {
      uint32_t v = ord[i];
      if (FV(v) > lambda || GV(v) > lambda) {
        if (lowk < BT(v) + GV(v)) {
          stop = 0;
          break;
        }
      }
    }
  }
#undef BT
#undef FV
#undef GV
  free(ord);
  return stop;
}

/* Wanted half-widths for the top-k task (section 5), from the pilot counts.
 * With v_1..v_n the pilot order and b0 the pilot estimate:
 *   i <= k: lambda_U = (b0(v_{i-1}) - b0(v_i))/2 (1 for i = 1),
 *           lambda_L = (b0(v_i) - b0(v_{i+1}))/2 (1 if there is no v_{i+1});
 *   a gap b0(v_i) - b0(v_{i+1}) < 2 lambda with i <= k ties v_i and v_{i+1}:
 *           both get lambda_L = lambda_U = lambda;
 *   the values of positions 1..k are clamped to [lambda, 1];
 *   i > k:  lambda (both) if tied, else lambda_L = 1 and
 *           lambda_U = clamp(b0(v_k) - lambda_L(v_k) - b0(v_i), lambda, 1). */
int or_topk_lambdas(uint32_t n, uint32_t k, const uint64_t *count0, uint64_t alpha, double lambda,
                    double *lam_l, double *lam_u) {
  uint32_t *ord = (uint32_t *)malloc((size_t)n * 4);
  uint8_t *tied = (uint8_t *)calloc(n, 1);
  if (!ord || !tied) {
    free(ord); free(tied);
    return OR_ENOMEM;
  }
  rank_order(n, count0, ord);
  double A = (double)alpha;
#define B0(pos) ((double)count0[ord[pos]] / A)
  for (uint32_t i = 0; i < k; ++i) {
    uint32_t v = ord[i];
    lam_u[v] = i == 0 ? 1.0 : (B0(i - 1) - B0(i)) / 2.0;
    lam_l[v] = i + 1 < n ? (B0(i) - B0(i + 1)) / 2.0 : 1.0;
  }
  for (uint32_t i = 0; i < k; ++i) {
    if (i + 1 < n && B0(i) - B0(i + 1) < 2.0 * lambda) {
      tied[i] = 1;
      tied[i + 1] = 1;
    }
  }
  for (uint32_t i = 0; i < k; ++i) {
    uint32_t v = ord[i];
    if (tied[i]) {
      lam_l[v] = lambda;
      lam_u[v] = lambda;
    }
    if (lam_l[v] < lambda) lam_l[v] = lambda;
    if (lam_l[v] > 1.0) lam_l[v] = 1.0;
    if (lam_u[v] < lambda) lam_u[v] = lambda;
    if (lam_u[v] > 1.0) lam_u[v] = 1.0;
  }
  double lk = B0(k - 1) - lam_l[ord[k - 1]];
  for (uint32_t i = k; i < n; ++i) {
    uint32_t v = ord[i];
    if (tied[i]) {
      lam_l[v] = lambda;
      lam_u[v] = lambda;
    } else {
      lam_l[v] = 1.0;
      double u = lk - B0(i);
      if (u < lambda) u = lambda;
      if (u > 1.0) u = 1.0;
      lam_u[v] = u;
    }
  }
#undef B0
  free(ord);
  free(tied);
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* The whole adaptive algorithm (Algorithm 1 with the batched check).          */
/* ------------------------------------------------------------------------- */
typedef struct {
  double epsilon, delta;
  uint32_t mode; /* 0 all nodes, 1 top-k */
  uint32_t k;
  uint64_t seed;
  uint64_t check_interval; /* 0: default rule */
  uint32_t vd_override;    /* 0: VD rule above */
  double c, balance_eps;   /* 0: 0.5 and 0.001 */
  double exact_vd_limit;   /* 0: 1e9 */
  int32_t threads;
  int32_t forward;         /* 1: forward BFS from s instead of the balanced search */
  int32_t edges;           /* 1: the betweenness of edges (items = edge ids) */
} or_params;

typedef struct {
  uint64_t tau, omega, alpha, interval, arcs, pilot_arcs;
  uint32_t vd, stop_rule; /* stop_rule 1: stopping condition, 0: tau reached omega */
  int32_t vd_exact;
  double C;
  /* arrays of one entry per item: node, or edge id with p->edges */
  uint64_t *count; /* main-phase hits */
  double *bc, *lower, *upper;
  double *L_l, *L_u;
  uint64_t *count0; /* pilot hits */
} or_result;

int or_run(const or_graph *g, const or_params *p, or_result *r) {
  if (!g || !p || !r || g->n < 2) return OR_EINVAL;
  if (!(p->epsilon > 0 && p->epsilon < 1 && p->delta > 0 && p->delta < 1)) return OR_EINVAL;
  /* the items whose betweenness is estimated: the nodes, or the edges */
  const uint64_t items = p->edges ? or_edge_count(g) : g->n;
  if (items < 1 || items > 0xFFFFFFFFull) return OR_EINVAL;
  if (p->mode == 1 && (p->k < 1 || p->k > items)) return OR_EINVAL;
  uint32_t n = (uint32_t)items;
  uint32_t *eid = NULL;
  if (p->edges) {
    eid = (uint32_t *)malloc((g->arcs ? g->arcs : 1) * sizeof(uint32_t));
    if (!eid) return OR_ENOMEM;
    int rc0 = or_edge_ids(g, eid);
    if (rc0) {
      free(eid);
      return rc0;
    }
  }
  double c = p->c > 0 ? p->c : 0.5;
  double eb = p->balance_eps > 0 ? p->balance_eps : 0.001;
  double lim = p->exact_vd_limit > 0 ? p->exact_vd_limit : 1e9;
  int rc;
  if (p->vd_override) {
    r->vd = p->vd_override;
    r->vd_exact = 0;
  } else if ((rc = or_vertex_diameter(g, lim, &r->vd, &r->vd_exact))) {
    return rc;
  }
  r->omega = p->edges ? or_omega_edges(p->epsilon, p->delta, r->vd, c)
                      : or_omega(p->epsilon, p->delta, r->vd, c);
  r->alpha = or_alpha(r->omega);
  r->interval = p->check_interval ? p->check_interval : or_default_interval(r->omega);

  uint64_t *cnt0 = r->count0 ? r->count0 : (uint64_t *)malloc((size_t)n * 8);
  double *lam_l = (double *)malloc((size_t)n * 8);
  double *lam_u = (double *)malloc((size_t)n * 8);
  double *Ll = r->L_l ? r->L_l : (double *)malloc((size_t)n * 8);
  double *Lu = r->L_u ? r->L_u : (double *)malloc((size_t)n * 8);
  uint64_t *cnt = r->count ? r->count : (uint64_t *)malloc((size_t)n * 8);
  if (!cnt0 || !lam_l || !lam_u || !Ll || !Lu || !cnt) return OR_ENOMEM;
  memset(cnt0, 0, (size_t)n * 8);
  memset(cnt, 0, (size_t)n * 8);

  /* pilot: phase 0, ids 0..alpha-1 */
  r->pilot_arcs = 0;
  if ((rc = p->edges ? add_edge_hits(g, p->seed, 0, 0, r->alpha, p->threads, p->forward, eid,
                                     cnt0, &r->pilot_arcs)
                    : add_hits(g, p->seed, 0, 0, r->alpha, p->threads, p->forward, cnt0,
                               &r->pilot_arcs)))
    return rc;
  if (p->mode == 1) {
    if ((rc = or_topk_lambdas(n, p->k, cnt0, r->alpha, p->epsilon, lam_l, lam_u))) return rc;
  } else {
    for (uint32_t v = 0; v < n; ++v) lam_l[v] = lam_u[v] = p->epsilon;
  }
  if ((rc = or_compute_delta(n, cnt0, r->alpha, r->omega, lam_l, lam_u, p->delta, eb, Ll, Lu,
                             &r->C)))
    return rc;

  /* main loop: phase 1, ids from 0, a check after every interval */
  uint64_t tau = 0;
  r->arcs = 0;
  r->stop_rule = 0;
  for (;;) {
    uint64_t b = r->omega - tau < r->interval ? r->omega - tau : r->interval;
    if ((rc = p->edges ? add_edge_hits(g, p->seed, 1, tau, b, p->threads, p->forward, eid, cnt,
                                       &r->arcs)
                      : add_hits(g, p->seed, 1, tau, b, p->threads, p->forward, cnt, &r->arcs)))
      return rc;
    tau += b;
    if (tau >= r->omega) break;
    int stop = p->mode == 1
                   ? or_stop_topk(n, p->k, cnt, tau, r->omega, p->epsilon, Ll, Lu)
                   : or_stop_all(n, cnt, tau, r->omega, p->epsilon, Ll, Lu);
    if (stop < 0) return stop;
    if (stop) {
      r->stop_rule = 1;
      break;
    }
  }
  r->tau = tau;

  /* estimates and intervals (Theorem 1) */
  double T = (double)tau, W = (double)r->omega;
  for (uint32_t v = 0; v < n; ++v) {
    double bt = (double)cnt[v] / T;
    if (r->bc) r->bc[v] = bt;
    double lo, hi;
    if (r->stop_rule) {
      lo = bt - or_f(bt, Ll[v], W, T);
      hi = bt + or_g(bt, Lu[v], W, T);
    } else {
      lo = bt - p->epsilon;
      hi = bt + p->epsilon;
    }
    if (r->lower) r->lower[v] = lo;
    if (r->upper) r->upper[v] = hi;
  }
  if (!r->count0) free(cnt0);
  if (!r->L_l) free(Ll);
  if (!r->L_u) free(Lu);
  if (!r->count) free(cnt);
  free(lam_l);
  free(lam_u);
  free(eid);
  return OR_OK;
}

/* Rank intervals for the top-k output (appendix tables): for every node v,
 * rank_lo = 1 + #{w != v : lower(w) >= upper(v)} and
 * rank_hi = #{w : upper(w) > lower(v)}. */
int or_rank_intervals(uint32_t n, const double *lower, const double *upper, uint32_t *rank_lo,
                      uint32_t *rank_hi) {
  for (uint32_t v = 0; v < n; ++v) {
    uint32_t lo = 1, hi = 0;
    for (uint32_t w = 0; w < n; ++w) {
      if (w != v && lower[w] >= upper[v]) lo++;
      if (upper[w] > lower[v]) hi++;
    }
    rank_lo[v] = lo;
    rank_hi[v] = hi;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Exact normalised betweenness (section 2 definition) by Brandes' algorithm:  */
/* bc(v) = 1/(n(n-1)) * sum over ordered pairs s != t, v not in {s,t}, of     */
/* sigma_st(v)/sigma_st.  Path counts in binary64 (small graphs only).         */
/* ------------------------------------------------------------------------- */
int or_brandes(const or_graph *g, double *bc) {
  uint32_t n = g->n;
  uint32_t *dist = (uint32_t *)malloc((size_t)n * 4);
  uint32_t *order = (uint32_t *)malloc((size_t)n * 4);
  double *sig = (double *)malloc((size_t)n * 8);
  double *dep = (double *)malloc((size_t)n * 8);
  if (!dist || !order || !sig || !dep) {
    free(dist); free(order); free(sig); free(dep);
    return OR_ENOMEM;
  }
  for (uint32_t v = 0; v < n; ++v) bc[v] = 0.0;
  for (uint32_t s = 0; s < n; ++s) {
    for (uint32_t v = 0; v < n; ++v) {
      dist[v] = UNSEEN;
      sig[v] = 0.0;
      dep[v] = 0.0;
    }
    size_t head = 0, tail = 0;
    dist[s] = 0;
    sig[s] = 1.0;
    order[tail++] = s;
    while (head < tail) {
      uint32_t u = order[head++];
      for (uint32_t j = g->row[u]; j < g->row[u + 1]; ++j) {
        uint32_t x = g->col[j];
        if (dist[x] == UNSEEN) {
          dist[x] = dist[u] + 1;
          order[tail++] = x;
        }
        if (dist[x] == dist[u] + 1) sig[x] += sig[u];
      }
    }
    /* dependencies, farthest first: delta(u) = sum over successors x of
     * sigma(u)/sigma(x) * (1 + delta(x)) */
    for (size_t k = tail; k-- > 0;) {
      uint32_t u = order[k];
      for (uint32_t j = g->row[u]; j < g->row[u + 1]; ++j) {
        uint32_t x = g->col[j];
        if (dist[x] == dist[u] + 1) dep[u] += sig[u] / sig[x] * (1.0 + dep[x]);
      }
      if (u != s) bc[u] += dep[u];
    }
  }
  double norm = 1.0 / ((double)n * (double)(n - 1));
  for (uint32_t v = 0; v < n; ++v) bc[v] *= norm;
  free(dist); free(order); free(sig); free(dep);
  return OR_OK;
}

/* Number of shortest s->t paths and their length, by one plain BFS with
 * arbitrary-precision counts (for the pins).  sigma is written as
 * little-endian words; returns the distance or -1 if unreachable. */
int64_t or_sigma_st(const or_graph *g, uint32_t s, uint32_t t, uint64_t *sigma_words,
                    uint32_t words) {
  uint32_t n = g->n;
  uint32_t *dist = (uint32_t *)malloc((size_t)n * 4);
  uint32_t *queue = (uint32_t *)malloc((size_t)n * 4);
  nat *sig = (nat *)calloc(n, sizeof(nat));
  int64_t res = -1;
  if (!dist || !queue || !sig) goto out;
  for (uint32_t v = 0; v < n; ++v) dist[v] = UNSEEN;
  size_t head = 0, tail = 0;
  dist[s] = 0;
  nat_set_u64(&sig[s], 1);
  queue[tail++] = s;
  while (head < tail) {
    uint32_t u = queue[head++];
    for (uint32_t j = g->row[u]; j < g->row[u + 1]; ++j) {
      uint32_t x = g->col[j];
      if (dist[x] == UNSEEN) {
        dist[x] = dist[u] + 1;
        queue[tail++] = x;
      }
      if (dist[x] == dist[u] + 1) nat_add(&sig[x], &sig[u]);
    }
  }
  if (dist[t] != UNSEEN) {
    res = dist[t];
    memset(sigma_words, 0, (size_t)words * 8);
    for (uint32_t k = 0; k < sig[t].len && k < words; ++k) sigma_words[k] = sig[t].d[k];
    if (sig[t].len > words) res = -2;
  }
out:
  if (sig)
    for (uint32_t v = 0; v < n; ++v) nat_free(&sig[v]);
  free(sig);
  free(dist);
  free(queue);
  return res;
}
