/* Greedy graph search (Algorithm 1) and approximate greedy search
 * (Algorithm 4, Supplementary C) in plain C, float64.  TEST INFRASTRUCTURE
 * ONLY: the tests and the CPU-baseline leg of the benchmark load it; the
 * library never does.  It shares no code with the HIP library.
 *
 * It is a second, compiled rendering of the oracle's search, written so that
 * the host's cores can be timed on the same workload: it follows the same
 * readings of the pseudo-code as the NumPy oracle (oracle/search.py):
 *
 *   - T holds at most ef_eff = max(ef, K) keys (d2, id), ordered
 *     lexicographically; a neighbour is admitted iff T is not full or its
 *     key is below the worst key of T, and the worst key is then evicted;
 *   - C is the set of unexpanded entries of T: each step expands the best
 *     unexpanded entry and the search stops when none is left;
 *   - Algorithm 4 screens the new neighbours of an expansion only when the
 *     number of expansions so far, the current one included, exceeds W and T
 *     is full at the start of the expansion; the bound is the worst key of T
 *     at that moment (one bound per expansion); a neighbour is skipped iff
 *     its estimate exceeds the bound (both squared); skipped neighbours stay
 *     visited; survivors get their exact distance and the normal admission.
 *
 * The estimate is Algorithm 3 taken from the definitions (Eq. 1 and Eq. 2):
 * for centre c, alpha_x = c.x / c.c (0 when c.c = 0), x_res = x - alpha_x c;
 * t_hat = cos(P q_res, P d_res) (0 when either projection is 0);
 * t = (t_hat - mu_hat) sigma / sigma_hat + mu + eps (scale 1 when
 * sigma_hat = 0, no clipping); L2 estimate
 * |q_proj - d_proj|^2 + |q_res|^2 + |d_res|^2 - 2 |q_res| |d_res| t.
 * Under the inner-product metric (Supplementary A) distances are -q.x and
 * the estimate is -(alpha_q alpha_d c.c + |q_res| |d_res| t).
 *
 * Every function is reentrant: the caller may run disjoint query ranges on
 * several threads at once. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { MODE_PLAIN = 0, MODE_FINGER = 1 };
enum { METRIC_L2 = 0, METRIC_IP = 2 };
enum { C_EXPANSIONS, C_EXACT, C_SCREENED, C_SKIPPED, C_VISITED, C_PREPS, C_COUNT };

/* squared L2 by direct differences, or -q.x */
static double distance(const double* q, const double* x, int m, int metric) {
  double s = 0.0;
  if (metric == METRIC_IP) {
    for (int j = 0; j < m; ++j) s += q[j] * x[j];
    return -s;
  }
  for (int j = 0; j < m; ++j) {
    const double d = q[j] - x[j];
    s += d * d;
  }
  return s;
}

static double dot(const double* a, const double* b, int m) {
  double s = 0.0;
  for (int j = 0; j < m; ++j) s += a[j] * b[j];
  return s;
}

/* Eq. 1 for x against centre c: returns alpha, writes x_res */
static double split(const double* x, const double* c, double cc, int m, double* res) {
  const double alpha = cc > 0.0 ? dot(x, c, m) / cc : 0.0;
  for (int j = 0; j < m; ++j) res[j] = x[j] - alpha * c[j];
  return alpha;
}

/* y = P x for P [r][m] row-major */
static void project(const double* P, int r, int m, const double* x, double* y) {
  for (int i = 0; i < r; ++i) y[i] = dot(P + (int64_t)i * m, x, m);
}

typedef struct {
  const double* P;
  int r;
  double mu, sigma, mu_hat, sigma_hat, eps;
} Tables;

/* Algorithm 3 for neighbour d of centre c; work holds 2m + 2r doubles */
static double estimate(const double* q, const double* c, const double* d, int m, int metric,
                       const Tables* t, double* work) {
  double* qr = work;
  double* dr = work + m;
  double* pq = work + 2 * m;
  double* pd = pq + t->r;
  const double cc = dot(c, c, m);
  const double aq = split(q, c, cc, m, qr);
  const double ad = split(d, c, cc, m, dr);
  project(t->P, t->r, m, qr, pq);
  project(t->P, t->r, m, dr, pd);
  const double den = sqrt(dot(pq, pq, t->r)) * sqrt(dot(pd, pd, t->r));
  const double t_hat = den > 0.0 ? dot(pq, pd, t->r) / den : 0.0;
  const double scale = t->sigma_hat > 0.0 ? t->sigma / t->sigma_hat : 1.0;
  const double tt = (t_hat - t->mu_hat) * scale + t->mu + t->eps;
  const double rq = sqrt(dot(qr, qr, m));
  const double rd = sqrt(dot(dr, dr, m));
  if (metric == METRIC_IP) return -(aq * ad * cc + rq * rd * tt);
  double proj = 0.0;
  for (int j = 0; j < m; ++j) {
    const double e = aq * c[j] - ad * c[j];
    proj += e * e;
  }
  return proj + rq * rq + rd * rd - 2.0 * rq * rd * tt;
}

/* T: keys sorted ascending by (d2, id), with an expanded flag */
typedef struct {
  double* d;
  int64_t* id;
  unsigned char* done;
  int len, cap;
} TopList;

static int key_less(double da, int64_t ia, double db, int64_t ib) {
  return da < db || (da == db && ia < ib);
}

static void admit(TopList* T, double d2, int64_t id) {
  if (T->len >= T->cap && !key_less(d2, id, T->d[T->len - 1], T->id[T->len - 1])) return;
  int pos = T->len < T->cap ? T->len : T->cap - 1; /* the evicted worst key makes room */
  while (pos > 0 && key_less(d2, id, T->d[pos - 1], T->id[pos - 1])) {
    T->d[pos] = T->d[pos - 1];
    T->id[pos] = T->id[pos - 1];
    T->done[pos] = T->done[pos - 1];
    --pos;
  }
  T->d[pos] = d2;
  T->id[pos] = id;
  T->done[pos] = 0;
  if (T->len < T->cap) ++T->len;
}

/* One query.  visit[] holds a stamp per node; ids equal to stamp are
 * visited.  Returns 0, or -1 on an invalid entry or neighbour id. */
static int search_one(const double* data, int64_t n, int m, const int32_t* graph, int deg,
                      const double* q, int64_t entry, int k, int mode, int metric,
                      int warmup, const Tables* tab, uint32_t* visit, uint32_t stamp,
                      TopList* T, int64_t* nbuf, double* work, int64_t* out_ids, double* out_d2,
                      int64_t* cnt, double* margin) {
  if (entry < 0 || entry >= n) return -1;
  for (int i = 0; i < C_COUNT; ++i) cnt[i] = 0;
  *margin = INFINITY;
  T->len = 0;
  admit(T, distance(q, data + entry * m, m, metric), entry);
  visit[entry] = stamp;
  int64_t visited = 1;
  cnt[C_EXACT] = 1;
  for (;;) {
    int b = 0;
    while (b < T->len && T->done[b]) ++b;
    if (b == T->len) break;
    T->done[b] = 1;
    const int64_t cur = T->id[b];
    ++cnt[C_EXPANSIONS];
    int nn = 0;
    for (int s = 0; s < deg; ++s) {
      const int64_t nb = graph[cur * deg + s];
      if (nb >= n) return -1;
      if (nb < 0 || visit[nb] == stamp) continue;
      visit[nb] = stamp;
      ++visited;
      nbuf[nn++] = nb;
    }
    if (nn == 0) continue;
    if (mode == MODE_FINGER && cnt[C_EXPANSIONS] > warmup && T->len >= T->cap) {
      const double ub2 = T->d[T->len - 1];
      cnt[C_SCREENED] += nn;
      ++cnt[C_PREPS];
      int keep = 0;
      for (int i = 0; i < nn; ++i) {
        const double est = estimate(q, data + cur * m, data + nbuf[i] * m, m, metric, tab, work);
        if (ub2 != 0.0) {
          const double mg = fabs(est - ub2) / fabs(ub2);
          if (mg < *margin) *margin = mg;
        }
        if (est > ub2)
          ++cnt[C_SKIPPED];
        else
          nbuf[keep++] = nbuf[i];
      }
      nn = keep;
    }
    for (int i = 0; i < nn; ++i) {
      admit(T, distance(q, data + nbuf[i] * m, m, metric), nbuf[i]);
      ++cnt[C_EXACT];
    }
  }
  cnt[C_VISITED] = visited;
  for (int j = 0; j < k; ++j) {
    out_ids[j] = j < T->len ? T->id[j] : -1;
    out_d2[j] = j < T->len ? T->d[j] : INFINITY;
  }
  return 0;
}

/* Queries [0, nq) of one batch, each from its own entry.  dm = {mu, sigma,
 * mu_hat, sigma_hat, eps}; P [r][m] and dm may be NULL in plain mode.
 * Outputs: ids [nq][k] and d2 [nq][k] (padded with -1 / +inf), counters
 * [nq][6] (expansions, exact, screened, skipped, visited, preps), margins
 * [nq] (smallest |est - ub2| / |ub2| over the screening decisions, +inf if
 * none).  Returns 0, -1 on invalid arguments, -2 when out of memory. */
int oracle_search_batch(const double* data, int64_t n, int32_t m, const int32_t* graph,
                        int32_t deg, const double* queries, int64_t nq, const int64_t* entries,
                        int32_t ef, int32_t k, int32_t mode, int32_t metric, int32_t warmup,
                        const double* P, int32_t r, const double* dm, int64_t* out_ids,
                        double* out_d2, int64_t* out_counters, double* out_margin) {
  if (n <= 0 || m <= 0 || deg <= 0 || nq < 0 || ef < 1 || k < 1) return -1;
  if (mode != MODE_PLAIN && mode != MODE_FINGER) return -1;
  if (metric != METRIC_L2 && metric != METRIC_IP) return -1;
  if (mode == MODE_FINGER && (P == NULL || dm == NULL || r < 1 || r > m)) return -1;
  Tables tab = {P, r, 0, 0, 0, 0, 0};
  if (dm) {
    tab.mu = dm[0];
    tab.sigma = dm[1];
    tab.mu_hat = dm[2];
    tab.sigma_hat = dm[3];
    tab.eps = dm[4];
  }
  const int ef_eff = ef > k ? ef : k;
  uint32_t* visit = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
  TopList T = {(double*)malloc(sizeof(double) * (size_t)ef_eff),
               (int64_t*)malloc(sizeof(int64_t) * (size_t)ef_eff),
               (unsigned char*)malloc((size_t)ef_eff), 0, ef_eff};
  int64_t* nbuf = (int64_t*)malloc(sizeof(int64_t) * (size_t)deg);
  double* work = (double*)malloc(sizeof(double) * (2 * (size_t)m + 2 * (size_t)(r > 0 ? r : 1)));
  int rc = 0;
  if (!visit || !T.d || !T.id || !T.done || !nbuf || !work) rc = -2;
  for (int64_t i = 0; i < nq && rc == 0; ++i)
    rc = search_one(data, n, m, graph, deg, queries + i * m, entries[i], k, mode, metric,
                    warmup, &tab, visit, (uint32_t)(i + 1), &T, nbuf, work, out_ids + i * k,
                    out_d2 + i * k, out_counters + i * C_COUNT, out_margin + i);
  free(visit);
  free(T.d);
  free(T.id);
  free(T.done);
  free(nbuf);
  free(work);
  return rc;
}
