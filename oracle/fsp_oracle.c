/*
 * fsp_oracle.c -- plain, slow, obviously-correct CPU oracle for the
 * permutation flow-shop lower bound and branch-and-bound.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file.  Only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark load it (through oracle/oracle.py).  It
 * shares no code, header, table or helper with the HIP path.
 *
 * What it computes (Chakroun & Melab, "An Adaptative Multi-GPU based
 * Branch-and-Bound", Sec. II):
 *   - Sec. II.B: n jobs visit machines M1..Mm in order, job j spends p[j][k]
 *     on machine k, one job per machine at a time, the same job order on every
 *     machine (permutation schedules), minimise the makespan.
 *   - Sec. II.B: a tree node is a scheduled prefix; branching appends one of
 *     the unscheduled jobs, so the root has n sons and there are n! leaves.
 *   - Sec. II.A: the four operators (branching, bounding, selection,
 *     elimination); a node whose lower bound cannot beat the best known
 *     schedule is eliminated.
 *   - Sec. V.D: the bound's cost is O(m^2 n log n).  The paper does not print
 *     the bound.  The reading used here (and written out step by step below)
 *     is the classical two-machine bound for the flow shop: for every pair of
 *     machines (k,l), k<l, relax all other machines to unbounded capacity,
 *     keep the work between k and l as a per-job time lag, and solve the
 *     resulting two-machine problem exactly by Johnson's rule on the
 *     lag-shifted times (Mitten's extension); add the earliest availability
 *     of each machine (head) and the smallest remaining work after machine l
 *     (tail).  m^2 pairs x a sort of n jobs is the O(m^2 n log n) the paper
 *     quotes.
 *
 * Everything is integer.  Intermediate values are held in int64 so that no
 * overflow question arises for any instance the library accepts.
 *
 * Where the paper is silent this oracle takes readings of its own; the ones
 * that change results are: the prune rule (LB >= UB eliminates, with a switch for
 * the literal "greater than"), children generated in ascending job id, the
 * Johnson tie-break (by job id, which cannot change the bound's value), and a
 * malformed node (duplicate id, id >= n, depth > n) bounding to -1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_INVALID (-1)

/* ------------------------------------------------------------------ */
/* Makespan recurrence (Sec. II.B, textbook permutation flow shop).     */
/* c[k] := completion time of the last scheduled job on machine k.      */
/* Appending job x: c[0] += p[x][0]; c[k] = max(c[k], c[k-1]) + p[x][k]. */
/* ------------------------------------------------------------------ */
static void front_of(const int32_t *p, int n, int m, const uint8_t *seq,
                     int len, int64_t *c) {
  (void)n;
  for (int k = 0; k < m; ++k) c[k] = 0;
  for (int i = 0; i < len; ++i) {
    int x = seq[i];
    c[0] += p[x * m + 0];
    for (int k = 1; k < m; ++k) {
      int64_t s = c[k] > c[k - 1] ? c[k] : c[k - 1];
      c[k] = s + p[x * m + k];
    }
  }
}

/* Completion time on every machine after the sequence seq[0..len). */
void orc_front(const int32_t *p, int n, int m, const uint8_t *seq, int len,
               int64_t *front_out) {
  front_of(p, n, m, seq, len, front_out);
}

/* Makespan of the (partial) sequence: completion on the last machine. */
int64_t orc_makespan(const int32_t *p, int n, int m, const uint8_t *seq,
                     int len) {
  int64_t c[256];
  front_of(p, n, m, seq, len, c);
  return c[m - 1];
}

/* ------------------------------------------------------------------ */
/* Two-machine relaxation for the pair (k,l) over a job subset.         */
/* ------------------------------------------------------------------ */

/* Time lag of job j between machines k and l: the work of j strictly
 * between them, which in the relaxation is a pure delay. */
static int64_t lag_of(const int32_t *p, int m, int j, int k, int l) {
  int64_t s = 0;
  for (int h = k + 1; h < l; ++h) s += p[j * m + h];
  return s;
}

typedef struct {
  int job;
  int64_t a; /* p[j][k] + lag   (Mitten's shifted first-machine time)  */
  int64_t b; /* p[j][l] + lag   (Mitten's shifted second-machine time) */
} jrec;

/* Johnson's rule on (a, b): jobs with a < b first, by a ascending; then the
 * jobs with a >= b, by b descending.  Equal keys are ordered by job id
 * (any order of equal keys is optimal, so the bound does not depend on it). */
static int johnson_cmp(const void *x, const void *y) {
  const jrec *u = (const jrec *)x, *v = (const jrec *)y;
  int gu = (u->a < u->b) ? 0 : 1;
  int gv = (v->a < v->b) ? 0 : 1;
  if (gu != gv) return gu - gv;
  if (gu == 0) {
    if (u->a != v->a) return u->a < v->a ? -1 : 1;
  } else {
    if (u->b != v->b) return u->b > v->b ? -1 : 1;
  }
  return u->job - v->job;
}

/* Johnson order, for pair (k,l), of the jobs listed in jobs[0..cnt).
 * Writes the ordered job ids to order_out. */
void orc_johnson_order(const int32_t *p, int n, int m, int k, int l,
                       const uint8_t *jobs, int cnt, uint8_t *order_out) {
  (void)n;
  jrec rec[256];
  for (int i = 0; i < cnt; ++i) {
    int j = jobs[i];
    int64_t L = lag_of(p, m, j, k, l);
    rec[i].job = j;
    rec[i].a = p[j * m + k] + L;
    rec[i].b = p[j * m + l] + L;
  }
  qsort(rec, (size_t)cnt, sizeof(jrec), johnson_cmp);
  for (int i = 0; i < cnt; ++i) order_out[i] = (uint8_t)rec[i].job;
}

/* ------------------------------------------------------------------ */
/* Lower bound of one node (Sec. II.B node; Sec. V.D complexity).       */
/* node = [d, s_1 .. s_d]: the scheduled prefix.                        */
/* pair_out (optional, m(m-1)/2 entries, pairs in lexicographic (k,l)   */
/* order): the per-pair bound, or -1 when U is empty.                   */
/* Returns the bound, or ORC_INVALID for a malformed node.              */
/* ------------------------------------------------------------------ */
int64_t orc_lower_bound_pairs(const int32_t *p, int n, int m,
                              const uint8_t *node, int64_t *pair_out) {
  int d = node[0];
  if (d > n) return ORC_INVALID;
  uint8_t used[256];
  memset(used, 0, sizeof(used));
  for (int i = 0; i < d; ++i) {
    int j = node[1 + i];
    if (j >= n || used[j]) return ORC_INVALID;
    used[j] = 1;
  }
  /* Step 1: front of the prefix on every machine. */
  int64_t F[256];
  front_of(p, n, m, node + 1, d, F);

  /* Step 2: the unscheduled set U. */
  uint8_t U[256];
  int u = 0;
  for (int j = 0; j < n; ++j)
    if (!used[j]) U[u++] = (uint8_t)j;

  int npairs = m * (m - 1) / 2;
  if (u == 0) {
    /* A complete schedule: its bound is its makespan. */
    if (pair_out)
      for (int q = 0; q < npairs; ++q) pair_out[q] = -1;
    return F[m - 1];
  }

  /* Step 3: heads.  Every unscheduled job starts on machine 0 no earlier
   * than F[0] and reaches machine k only after its work on machines 0..k-1;
   * machine k itself is busy until F[k]. */
  int64_t r[256];
  for (int k = 0; k < m; ++k) {
    int64_t best = -1;
    for (int i = 0; i < u; ++i) {
      int j = U[i];
      int64_t before = 0;
      for (int h = 0; h < k; ++h) before += p[j * m + h];
      if (best < 0 || before < best) best = before;
    }
    int64_t e = F[0] + best;
    r[k] = F[k] > e ? F[k] : e;
  }
  /* Step 4: tails.  Whichever job finishes last on machine l still needs its
   * work on machines l+1..m-1. */
  int64_t q[256];
  for (int l = 0; l < m; ++l) {
    int64_t best = -1;
    for (int i = 0; i < u; ++i) {
      int j = U[i];
      int64_t after = 0;
      for (int h = l + 1; h < m; ++h) after += p[j * m + h];
      if (best < 0 || after < best) best = after;
    }
    q[l] = best;
  }

  /* Step 5: every machine pair, Johnson order with Mitten lags. */
  int64_t lb = -1;
  int pi = 0;
  uint8_t order[256];
  for (int k = 0; k < m; ++k) {
    for (int l = k + 1; l < m; ++l, ++pi) {
      orc_johnson_order(p, n, m, k, l, U, u, order);
      int64_t tk = r[k], tl = r[l];
      for (int i = 0; i < u; ++i) {
        int j = order[i];
        tk += p[j * m + k];
        int64_t arrive = tk + lag_of(p, m, j, k, l);
        tl = (tl > arrive ? tl : arrive) + p[j * m + l];
      }
      int64_t v = tl + q[l];
      if (pair_out) pair_out[pi] = v;
      if (v > lb) lb = v;
    }
  }
  return lb;
}

int64_t orc_lower_bound(const int32_t *p, int n, int m, const uint8_t *node) {
  return orc_lower_bound_pairs(p, n, m, node, NULL);
}

/* ------------------------------------------------------------------ */
/* One-machine bound of a node (Sec. VI names other lower bounds as    */
/* future work; this is the classic cheaper one): on each machine h,    */
/* every unscheduled job passes h no earlier than the head of h, one    */
/* after the other, and whichever passes last still has the smallest    */
/* tail of h ahead of it.  Bound = max over h of head + remaining work  */
/* + tail; the makespan for a complete node; ORC_INVALID for a          */
/* malformed one.                                                       */
/* ------------------------------------------------------------------ */
int64_t orc_lower_bound_one_machine(const int32_t *p, int n, int m,
                                    const uint8_t *node) {
  const int depth = node[0];
  if (depth > n) return ORC_INVALID;
  uint8_t seen[256];
  memset(seen, 0, sizeof(seen));
  for (int i = 1; i <= depth; ++i) {
    const int job = node[i];
    if (job >= n || seen[job]) return ORC_INVALID;
    seen[job] = 1;
  }
  int64_t front[256];
  front_of(p, n, m, node + 1, depth, front);
  if (depth == n) return front[m - 1];
  int64_t best = 0;
  for (int h = 0; h < m; ++h) {
    int64_t work = 0, min_before = -1, min_after = -1;
    for (int job = 0; job < n; ++job) {
      if (seen[job]) continue;
      int64_t before = 0, after = 0;
      for (int g = 0; g < m; ++g) {
        if (g < h) before += p[job * m + g];
        if (g > h) after += p[job * m + g];
      }
      work += p[job * m + h];
      if (min_before < 0 || before < min_before) min_before = before;
      if (min_after < 0 || after < min_after) min_after = after;
    }
    /* head of h: machine h is free at front[h]; the first unscheduled job
     * leaves machine 0 no earlier than front[0] and then needs its work
     * on machines 0..h-1 */
    int64_t head = front[0] + min_before;
    if (front[h] > head) head = front[h];
    const int64_t v = head + work + min_after;
    if (v > best) best = v;
  }
  return best;
}

/* ------------------------------------------------------------------ */
/* Bounding a pool (Sec. III: every sub-problem of the pool is bounded  */
/* independently).  Records are `stride` bytes: [d, s_1..s_d, ...].     */
/* nthreads > 1 splits the pool into equal contiguous parts.            */
/* ------------------------------------------------------------------ */
typedef struct {
  const int32_t *p;
  int n, m, stride;
  const uint8_t *nodes;
  int64_t begin, end;
  int32_t *out;
  int one_machine; /* 1: the one-machine bound instead of the pair bound */
} pool_job;

static void *pool_worker(void *arg) {
  pool_job *w = (pool_job *)arg;
  for (int64_t i = w->begin; i < w->end; ++i) {
    const uint8_t *rec = w->nodes + i * (int64_t)w->stride;
    w->out[i] = (int32_t)(w->one_machine
                              ? orc_lower_bound_one_machine(w->p, w->n, w->m, rec)
                              : orc_lower_bound(w->p, w->n, w->m, rec));
  }
  return NULL;
}

static void bound_pool_with(const int32_t *p, int n, int m, const uint8_t *nodes,
                            int stride, int64_t count, int32_t *lb_out, int nthreads,
                            int one_machine);

void orc_bound_pool(const int32_t *p, int n, int m, const uint8_t *nodes,
                    int stride, int64_t count, int32_t *lb_out, int nthreads) {
  bound_pool_with(p, n, m, nodes, stride, count, lb_out, nthreads, 0);
}

void orc_bound_pool_one_machine(const int32_t *p, int n, int m, const uint8_t *nodes,
                                int stride, int64_t count, int32_t *lb_out,
                                int nthreads) {
  bound_pool_with(p, n, m, nodes, stride, count, lb_out, nthreads, 1);
}

static void bound_pool_with(const int32_t *p, int n, int m, const uint8_t *nodes,
                            int stride, int64_t count, int32_t *lb_out, int nthreads,
                            int one_machine) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pool_job jobs[256];
  pthread_t th[256];
  int64_t per = (count + nthreads - 1) / nthreads;
  int started = 0;
  for (int t = 0; t < nthreads; ++t) {
    int64_t b = t * per, e = b + per;
    if (e > count) e = count;
    if (b >= e) break;
    jobs[t] = (pool_job){p, n, m, stride, nodes, b, e, lb_out, one_machine};
    if (nthreads == 1) {
      pool_worker(&jobs[t]);
    } else {
      pthread_create(&th[t], NULL, pool_worker, &jobs[t]);
      ++started;
    }
  }
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------ */
/* NEH insertion heuristic (initial upper bound; not part of the paper, */
/* which seeds its runs from a list of sub-problems instead).           */
/* Jobs by total work descending (ties: smaller id first); insert each  */
/* at the position 0..len minimising the partial makespan (earliest     */
/* position on ties).                                                   */
/* ------------------------------------------------------------------ */
int64_t orc_neh(const int32_t *p, int n, int m, uint8_t *perm_out) {
  int idx[256];
  int64_t tot[256];
  for (int j = 0; j < n; ++j) {
    idx[j] = j;
    tot[j] = 0;
    for (int k = 0; k < m; ++k) tot[j] += p[j * m + k];
  }
  /* insertion sort: total descending, id ascending */
  for (int a = 1; a < n; ++a) {
    int x = idx[a], b = a - 1;
    while (b >= 0 && (tot[idx[b]] < tot[x] ||
                      (tot[idx[b]] == tot[x] && idx[b] > x))) {
      idx[b + 1] = idx[b];
      --b;
    }
    idx[b + 1] = x;
  }
  uint8_t seq[256], trial[256];
  int len = 0;
  seq[len++] = (uint8_t)idx[0];
  for (int a = 1; a < n; ++a) {
    int x = idx[a];
    int best_pos = 0;
    int64_t best = -1;
    for (int pos = 0; pos <= len; ++pos) {
      int t = 0;
      for (int i = 0; i < pos; ++i) trial[t++] = seq[i];
      trial[t++] = (uint8_t)x;
      for (int i = pos; i < len; ++i) trial[t++] = seq[i];
      int64_t c = orc_makespan(p, n, m, trial, t);
      if (best < 0 || c < best) {
        best = c;
        best_pos = pos;
      }
    }
    for (int i = len; i > best_pos; --i) seq[i] = seq[i - 1];
    seq[best_pos] = (uint8_t)x;
    ++len;
  }
  memcpy(perm_out, seq, (size_t)n);
  return orc_makespan(p, n, m, seq, n);
}

/* ------------------------------------------------------------------ */
/* Brute force: minimum makespan over all n! permutations (Sec. II.B:   */
/* the search space is the n! schedules).  Lexicographic enumeration;   */
/* the first permutation reaching the minimum is returned.              */
/* ------------------------------------------------------------------ */
static int next_permutation(uint8_t *a, int n) {
  int i = n - 2;
  while (i >= 0 && a[i] >= a[i + 1]) --i;
  if (i < 0) return 0;
  int j = n - 1;
  while (a[j] <= a[i]) --j;
  uint8_t t = a[i];
  a[i] = a[j];
  a[j] = t;
  for (int x = i + 1, y = n - 1; x < y; ++x, --y) {
    t = a[x];
    a[x] = a[y];
    a[y] = t;
  }
  return 1;
}

int64_t orc_brute_force(const int32_t *p, int n, int m, uint8_t *perm_out) {
  uint8_t a[256];
  for (int j = 0; j < n; ++j) a[j] = (uint8_t)j;
  int64_t best = -1;
  do {
    int64_t c = orc_makespan(p, n, m, a, n);
    if (best < 0 || c < best) {
      best = c;
      memcpy(perm_out, a, (size_t)n);
    }
  } while (next_permutation(a, n));
  return best;
}

/* Minimum makespan over all completions of the node [d, s_1..s_d]
 * (brute force over the (n-d)! orders of the unscheduled jobs). */
int64_t orc_best_completion(const int32_t *p, int n, int m,
                            const uint8_t *node) {
  int d = node[0];
  uint8_t used[256], seq[256], rest[256];
  memset(used, 0, sizeof(used));
  for (int i = 0; i < d; ++i) {
    seq[i] = node[1 + i];
    used[seq[i]] = 1;
  }
  int u = 0;
  for (int j = 0; j < n; ++j)
    if (!used[j]) rest[u++] = (uint8_t)j;
  int64_t best = -1;
  do {
    memcpy(seq + d, rest, (size_t)u);
    int64_t c = orc_makespan(p, n, m, seq, n);
    if (best < 0 || c < best) best = c;
  } while (next_permutation(rest, u));
  return best;
}

/* ------------------------------------------------------------------ */
/* Sequential depth-first branch-and-bound: the paper's CPU baseline,   */
/* a serial B&B on one core (Sec. V.C), with the four operators of      */
/* Sec. II.A.                                                           */
/*   UB := ub_in if > 0, else NEH.  Bound the root.                     */
/*   Pop the most recently pushed node; if it can no longer beat UB it   */
/*   is eliminated; else branch it: children v||j for j in U ascending,  */
/*   each bounded.  A complete child with LB < UB is a better schedule:  */
/*   UB := LB.  An incomplete child is kept if it can still beat UB.     */
/*   Kept children are pushed so that the smallest j is popped first.    */
/* rule 0: eliminate when LB >= UB.  rule 1: eliminate when LB > UB      */
/* (the paper's literal wording); a leaf must still be strictly better.  */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t nodes_bounded;  /* every bound evaluation, root included */
  int64_t nodes_branched; /* nodes whose children were generated */
  int64_t nodes_pruned;   /* children discarded + popped nodes eliminated */
  int64_t leaves;         /* complete schedules bounded */
  int32_t found;          /* 1 if a schedule better than the initial UB */
  int32_t root_lb;
  int32_t complete;       /* 1 if the tree was exhausted (optimum proven) */
  int32_t pad;
} orc_stats;

static int keeps(int rule, int64_t lb, int64_t ub) {
  return rule == 1 ? (lb <= ub) : (lb < ub);
}

/* The bound of a node under a per-depth choice (Sec. VI: other lower
 * bounds): a node of depth d, 0 < d < n, whose bit d is set in lb1_mask (8
 * words, bit d of word d / 32) takes the one-machine bound; every other node
 * (the root, complete schedules, unset depths, or no mask) the two-machine
 * bound. */
static int64_t bound_at_depth(const int32_t *p, int n, int m, const uint8_t *node,
                              const uint32_t *lb1_mask) {
  const int d = node[0];
  if (lb1_mask && d > 0 && d < n && ((lb1_mask[d >> 5] >> (d & 31)) & 1u))
    return orc_lower_bound_one_machine(p, n, m, node);
  return orc_lower_bound(p, n, m, node);
}

int64_t orc_bnb_choice(const int32_t *p, int n, int m, int64_t ub_in, int rule,
                       int64_t max_bounded, const uint32_t *lb1_mask, uint8_t *perm_out,
                       orc_stats *st) {
  /* max_bounded > 0 stops the search once that many bounds were evaluated
   * (complete = 0); the returned UB is then only an upper bound. */
  memset(st, 0, sizeof(*st));
  int64_t ub;
  if (ub_in > 0) {
    ub = ub_in;
    for (int j = 0; j < n; ++j) perm_out[j] = (uint8_t)j;
  } else {
    ub = orc_neh(p, n, m, perm_out);
  }
  /* Each stack entry: a node record (n+1 bytes) and its bound. */
  int rec = n + 1;
  int64_t cap = (int64_t)n * n + 16;
  uint8_t *stk = (uint8_t *)malloc((size_t)(cap * rec));
  int64_t *slb = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
  uint8_t root[257];
  memset(root, 0, sizeof(root));
  int64_t rlb = orc_lower_bound(p, n, m, root);
  st->nodes_bounded = 1;
  st->root_lb = (int32_t)rlb;
  int64_t top = 0;
  if (n == 0) {
    st->complete = 1;
    free(stk);
    free(slb);
    return ub;
  }
  if (keeps(rule, rlb, ub)) {
    memcpy(stk, root, (size_t)rec);
    slb[0] = rlb;
    top = 1;
  } else {
    st->nodes_pruned++;
  }
  uint8_t child[257];
  uint8_t kept[256][257];
  int64_t kept_lb[256];
  while (top > 0) {
    if (max_bounded > 0 && st->nodes_bounded >= max_bounded) break;
    --top;
    uint8_t *v = stk + top * rec;
    int64_t vlb = slb[top];
    if (!keeps(rule, vlb, ub)) { /* UB improved since it was kept */
      st->nodes_pruned++;
      continue;
    }
    int d = v[0];
    uint8_t used[256];
    memset(used, 0, sizeof(used));
    for (int i = 0; i < d; ++i) used[v[1 + i]] = 1;
    st->nodes_branched++;
    int nk = 0;
    for (int j = 0; j < n; ++j) {
      if (used[j]) continue;
      memcpy(child, v, (size_t)rec);
      child[0] = (uint8_t)(d + 1);
      child[1 + d] = (uint8_t)j;
      int64_t clb = bound_at_depth(p, n, m, child, lb1_mask);
      st->nodes_bounded++;
      if (d + 1 == n) {
        st->leaves++;
        if (clb < ub) {
          ub = clb;
          memcpy(perm_out, child + 1, (size_t)n);
          st->found = 1;
        } else {
          st->nodes_pruned++;
        }
      } else if (keeps(rule, clb, ub)) {
        memcpy(kept[nk], child, (size_t)rec);
        kept_lb[nk] = clb;
        ++nk;
      } else {
        st->nodes_pruned++;
      }
    }
    for (int i = nk - 1; i >= 0; --i) {
      memcpy(stk + top * rec, kept[i], (size_t)rec);
      slb[top] = kept_lb[i];
      ++top;
    }
  }
  st->complete = (top == 0);
  free(stk);
  free(slb);
  return ub;
}

/* The search with the two-machine bound at every depth. */
int64_t orc_bnb(const int32_t *p, int n, int m, int64_t ub_in, int rule,
                int64_t max_bounded, uint8_t *perm_out, orc_stats *st) {
  return orc_bnb_choice(p, n, m, ub_in, rule, max_bounded, NULL, perm_out, st);
}
