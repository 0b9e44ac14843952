/*
 * CPU oracle for single-source shortest paths and delta-stepping.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library path links, loads or calls
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline do. It shares no code, header or table with the GPU library.
 *
 * What is computed (Sec. III of the paper, problem statement): for a directed
 * graph with positive edge weights and a source s, d(v) = the minimum over all
 * directed paths s = v0 -> ... -> vk = v of the path weight, the path weight
 * being the left fold x0 = 0, xj = x(j-1) (+) w(v(j-1), vj). The addition (+)
 * follows the weight type:
 *   ORC_U32  exact integer addition; a distance above 2^32 - 2 cannot be
 *            represented (2^32 - 1 encodes "unreachable") and is an overflow;
 *   ORC_F32  binary32 addition rounded to nearest-even (the fp32 arithmetic of
 *            an fp32 edge weight); a sum rounding to +inf is an overflow;
 *   ORC_F64  binary64 addition rounded to nearest-even (the paper's GrB_FP64).
 * d(s) = 0 and d(v) = infinity when no path exists.
 *
 * All distances are held in double internally. For ORC_U32 every value that is
 * kept is an integer below 2^33, exact in double; for ORC_F32 every value is a
 * binary32 number (exact in double) and each addition is performed in float.
 *
 * Functions:
 *   orc_dijkstra      textbook Dijkstra with a binary heap (lazy deletion);
 *   orc_delta_la      the paper's linear-algebra delta-stepping (Fig. 1 left),
 *                     dense vectors, synchronous request vector, with a trace;
 *   orc_delta_sets    Meyer-Sanders delta-stepping with explicit buckets and
 *                     the relax procedure (Sec. III-C, Fig. 1 right);
 *   orc_bellman_ford  brute-force Bellman-Ford (n rounds over all edges);
 *   orc_certify       O(m) optimality certificate of a candidate distance vector;
 *   orc_sp_gradient   dL/dw by reverse accumulation over the shortest-path tree;
 *   orc_dijkstra_many orc_dijkstra from many sources on host threads (timing aid).
 *
 * Build: gcc -O2 -fPIC -shared -pthread -ffp-contract=off -fno-fast-math (x86-64 SSE
 * arithmetic: float and double operations are rounded once, no excess precision).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_U32 = 0, ORC_F32 = 1, ORC_F64 = 2 };
enum {
  ORC_OK = 0,
  ORC_OVERFLOW = 1,       /* some reachable vertex has an unrepresentable distance */
  ORC_BADARG = 2,
  ORC_NOMEM = 3,
  ORC_CLOSED_BUCKET = 4,  /* delta_sets: a vertex fell into an already closed bucket */
};

/* certificate verdicts */
enum {
  CERT_OK = 0,
  CERT_SOURCE = 1,       /* d(s) is not +0 */
  CERT_VALUE = 2,        /* a value that no path weight can take (NaN, negative, -0.0, 2^32-1 misuse) */
  CERT_FEASIBLE = 3,     /* an edge (u,v) with d(u) finite and d(u) (+) w < d(v) */
  CERT_OVERFLOW = 4,     /* d(u) finite, d(u) (+) w overflows and d(v) is infinite */
  CERT_TIGHT = 5,        /* a finite d(v) not reached from s through tight edges */
};

#define U32_MAX_DIST 4294967294.0 /* largest representable u32 distance */

static double weight_of(int kind, const void *w, int64_t e) {
  switch (kind) {
    case ORC_U32: return (double)((const uint32_t *)w)[e];
    case ORC_F32: return (double)((const float *)w)[e];
    default: return ((const double *)w)[e];
  }
}

/* x (+) w in the weight type's arithmetic. Returns +inf and sets *ovf when the
 * sum cannot be represented. x is finite and non-negative. */
static double plus(int kind, double x, double w, int *ovf) {
  *ovf = 0;
  if (kind == ORC_U32) {
    double s = x + w; /* both integers < 2^33: exact */
    if (s > U32_MAX_DIST) { *ovf = 1; return INFINITY; }
    return s;
  }
  if (kind == ORC_F32) {
    float a = (float)x, b = (float)w; /* exact: both are binary32 values */
    float s = a + b;                   /* one binary32 rounding */
    if (isinf(s)) { *ovf = 1; return INFINITY; }
    return (double)s;
  }
  double s = x + w;
  if (isinf(s)) { *ovf = 1; return INFINITY; }
  return s;
}

static void store_dist(int kind, void *out, int64_t v, double d) {
  switch (kind) {
    case ORC_U32: ((uint32_t *)out)[v] = isinf(d) ? 0xFFFFFFFFu : (uint32_t)d; break;
    case ORC_F32: ((float *)out)[v] = (float)d; break;
    default: ((double *)out)[v] = d; break;
  }
}

static double load_dist(int kind, const void *in, int64_t v) {
  switch (kind) {
    case ORC_U32: {
      uint32_t x = ((const uint32_t *)in)[v];
      return x == 0xFFFFFFFFu ? INFINITY : (double)x;
    }
    case ORC_F32: return (double)((const float *)in)[v];
    default: return ((const double *)in)[v];
  }
}

static int check_args(int64_t n, const int64_t *rp, const int32_t *col, int32_t src) {
  if (n <= 0 || !rp || src < 0 || src >= n) return 0;
  if (rp[0] != 0) return 0;
  for (int64_t u = 0; u < n; ++u)
    if (rp[u + 1] < rp[u]) return 0;
  for (int64_t e = 0; e < rp[n]; ++e)
    if (!col || col[e] < 0 || col[e] >= n) return 0;
  return 1;
}

/* after a run with candidate dropping: an overflow happened at v and v stayed
 * infinite means v is reachable only through unrepresentable sums. */
static int overflow_verdict(int64_t n, const double *d, const unsigned char *ovf_at) {
  for (int64_t v = 0; v < n; ++v)
    if (ovf_at[v] && isinf(d[v])) return ORC_OVERFLOW;
  return ORC_OK;
}

/* ------------------------------------------------------------ Dijkstra */

typedef struct { double key; int64_t v; } heap_item;

static void heap_push(heap_item *h, int64_t *len, double key, int64_t v) {
  int64_t i = (*len)++;
  h[i].key = key; h[i].v = v;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].key <= h[i].key) break;
    heap_item t = h[p]; h[p] = h[i]; h[i] = t;
    i = p;
  }
}

static heap_item heap_pop(heap_item *h, int64_t *len) {
  heap_item top = h[0];
  h[0] = h[--(*len)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    if (l < *len && h[l].key < h[s].key) s = l;
    if (r < *len && h[r].key < h[s].key) s = r;
    if (s == i) break;
    heap_item t = h[s]; h[s] = h[i]; h[i] = t;
    i = s;
  }
  return top;
}

int orc_dijkstra(int64_t n, const int64_t *rp, const int32_t *col, const void *w, int kind, int32_t src,
                 void *dist_out) {
  if (!check_args(n, rp, col, src) || kind < 0 || kind > 2) return ORC_BADARG;
  int64_t m = rp[n];
  double *d = malloc(sizeof(double) * n);
  unsigned char *done = calloc(n, 1), *ovf_at = calloc(n, 1);
  heap_item *h = malloc(sizeof(heap_item) * (m + 1));
  if (!d || !done || !ovf_at || !h) { free(d); free(done); free(ovf_at); free(h); return ORC_NOMEM; }
  for (int64_t v = 0; v < n; ++v) d[v] = INFINITY;
  int64_t len = 0;
  d[src] = 0.0;
  heap_push(h, &len, 0.0, src);
  while (len > 0) {
    heap_item it = heap_pop(h, &len);
    int64_t u = it.v;
    if (done[u] || it.key != d[u]) continue; /* stale entry */
    done[u] = 1;
    for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
      int64_t v = col[e];
      int ovf;
      double c = plus(kind, d[u], weight_of(kind, w, e), &ovf);
      if (ovf) { ovf_at[v] = 1; continue; }
      if (c < d[v]) { d[v] = c; heap_push(h, &len, c, v); }
    }
  }
  int rc = overflow_verdict(n, d, ovf_at);
  for (int64_t v = 0; v < n; ++v) store_dist(kind, dist_out, v, d[v]);
  free(d); free(done); free(ovf_at); free(h);
  return rc;
}

/* ------------------------------------------------------------ buckets */

/* exact tests of t >= k*delta and t < k*delta for real t, delta > 0, integer k:
 * fma(-k, delta, t) is t - k*delta rounded once, which keeps the exact sign. */
static int ge_multiple(double t, double k, double delta) { return fma(-k, delta, t) >= 0.0; }
static int lt_multiple(double t, double k, double delta) { return fma(-k, delta, t) < 0.0; }

/* bucket index floor(t / delta) for finite t >= 0, exact */
static int64_t bucket_of(double t, double delta) {
  double k = floor(t / delta);
  while (k > 0 && lt_multiple(t, k, delta)) k -= 1.0;
  while (ge_multiple(t, k + 1.0, delta)) k += 1.0;
  return (int64_t)k;
}

int64_t orc_bucket_of(double t, double delta) { return bucket_of(t, delta); }

/* the threshold value used for the light/heavy split in the weight type */
static double split_threshold(int kind, double delta) {
  if (kind == ORC_F32) return (double)(float)delta;
  return delta;
}

/* light iff 0 < w <= delta, heavy iff w > delta (Sec. III-A; A_L = A o (0 < A <= delta),
 * A_H = A o (A > delta), Sec. IV-A) */
static int is_light(double w, double delta) { return w > 0.0 && w <= delta; }
static int is_heavy(double w, double delta) { return w > delta; }

typedef struct {
  int64_t cap;            /* capacity of the per-bucket arrays below */
  int64_t nbuckets;       /* buckets whose S was non-empty */
  int64_t *bucket;        /* [cap] index i of each such bucket */
  int64_t *s_size;        /* [cap] |S_i| */
  int64_t *inner;         /* [cap] light-phase iterations spent in bucket i */
  int64_t outer_iters;    /* outer iterations, empty buckets included */
  int64_t light_relax;    /* light edges scanned, summed over light phases */
  int64_t heavy_relax;    /* heavy edges scanned, summed over heavy phases */
  int64_t late_requests;  /* heavy requests that fell below (i+1)*delta (never in exact arithmetic) */
  int64_t *s_bucket;      /* [n] or NULL: bucket i in which v entered S (-1 if never) */
  int64_t s_conflicts;    /* a vertex entering S in two different buckets */
} orc_trace;

static void trace_bucket(orc_trace *tr, int64_t i, int64_t ssize, int64_t inner) {
  if (!tr || ssize == 0) return;
  if (tr->nbuckets < tr->cap && tr->bucket) {
    tr->bucket[tr->nbuckets] = i;
    tr->s_size[tr->nbuckets] = ssize;
    tr->inner[tr->nbuckets] = inner;
  }
  tr->nbuckets++;
}

static void trace_s_member(orc_trace *tr, int64_t v, int64_t i) {
  if (!tr || !tr->s_bucket) return;
  if (tr->s_bucket[v] >= 0 && tr->s_bucket[v] != i) tr->s_conflicts++;
  tr->s_bucket[v] = i;
}

/*
 * The linear-algebra formulation (Fig. 1 left; Sec. IV), in its own order:
 *   A_L = A o (0 < A <= delta), A_H = A o (A > delta)
 *   t = inf, t[s] = 0, i = 0
 *   while (t >= i*delta) != 0:                       -- over finite entries
 *     S = 0
 *     tB = (i*delta <= t < (i+1)*delta)
 *     while tB != 0:
 *       tReq = A_L^T (t o tB)                          -- min-plus, absent = inf
 *       S = (S + tB) > 0
 *       tB = (i*delta <= tReq < (i+1)*delta) o (tReq < t)   -- before the min
 *       t = min(t, tReq)
 *     tReq = A_H^T (t o S)
 *     t = min(t, tReq)
 *     i = i + 1
 * Every vector is dense; "absent" entries are +inf.
 */
int orc_delta_la(int64_t n, const int64_t *rp, const int32_t *col, const void *w, int kind, double delta,
                 int32_t src, void *dist_out, orc_trace *tr) {
  if (!check_args(n, rp, col, src) || kind < 0 || kind > 2 || !(delta > 0) || isinf(delta)) return ORC_BADARG;
  double dl = split_threshold(kind, delta);
  double *t = malloc(sizeof(double) * n), *treq = malloc(sizeof(double) * n);
  unsigned char *tb = malloc(n), *S = malloc(n), *ovf_at = calloc(n, 1);
  if (!t || !treq || !tb || !S || !ovf_at) {
    free(t); free(treq); free(tb); free(S); free(ovf_at); return ORC_NOMEM;
  }
  if (tr) {
    tr->nbuckets = tr->outer_iters = tr->light_relax = tr->heavy_relax = tr->late_requests = 0;
    tr->s_conflicts = 0;
    if (tr->s_bucket) for (int64_t v = 0; v < n; ++v) tr->s_bucket[v] = -1;
  }
  for (int64_t v = 0; v < n; ++v) t[v] = INFINITY;
  t[src] = 0.0;
  double i = 0.0;
  for (;;) {
    /* outer test: some finite t[v] >= i*delta */
    int more = 0;
    for (int64_t v = 0; v < n && !more; ++v) more = !isinf(t[v]) && ge_multiple(t[v], i, dl);
    if (!more) break;
    if (tr) tr->outer_iters++;
    memset(S, 0, n);
    for (int64_t v = 0; v < n; ++v)
      tb[v] = !isinf(t[v]) && ge_multiple(t[v], i, dl) && lt_multiple(t[v], i + 1.0, dl);
    int64_t inner = 0;
    for (;;) {
      int any = 0;
      for (int64_t v = 0; v < n && !any; ++v) any = tb[v];
      if (!any) break;
      inner++;
      /* tReq = A_L^T (t o tB) */
      for (int64_t v = 0; v < n; ++v) treq[v] = INFINITY;
      for (int64_t u = 0; u < n; ++u) {
        if (!tb[u]) continue;
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
          double we = weight_of(kind, w, e);
          if (!is_light(we, dl)) continue;
          if (tr) tr->light_relax++;
          int ovf;
          double c = plus(kind, t[u], we, &ovf);
          if (ovf) { ovf_at[col[e]] = 1; continue; }
          if (c < treq[col[e]]) treq[col[e]] = c;
        }
      }
      /* S = (S + tB) > 0 */
      for (int64_t v = 0; v < n; ++v)
        if (tb[v]) { S[v] = 1; trace_s_member(tr, v, (int64_t)i); }
      /* tB = (i*delta <= tReq < (i+1)*delta) o (tReq < t), then t = min(t, tReq) */
      for (int64_t v = 0; v < n; ++v)
        tb[v] = !isinf(treq[v]) && ge_multiple(treq[v], i, dl) && lt_multiple(treq[v], i + 1.0, dl) &&
                treq[v] < t[v];
      for (int64_t v = 0; v < n; ++v)
        if (treq[v] < t[v]) t[v] = treq[v];
    }
    /* heavy phase: tReq = A_H^T (t o S), t = min(t, tReq) */
    for (int64_t v = 0; v < n; ++v) treq[v] = INFINITY;
    int64_t ssize = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (!S[u]) continue;
      ssize++;
      for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
        double we = weight_of(kind, w, e);
        if (!is_heavy(we, dl)) continue;
        if (tr) tr->heavy_relax++;
        int ovf;
        double c = plus(kind, t[u], we, &ovf);
        if (ovf) { ovf_at[col[e]] = 1; continue; }
        if (c < treq[col[e]]) treq[col[e]] = c;
      }
    }
    for (int64_t v = 0; v < n; ++v) {
      if (treq[v] < t[v]) {
        if (tr && lt_multiple(treq[v], i + 1.0, dl)) tr->late_requests++;
        t[v] = treq[v];
      }
    }
    trace_bucket(tr, (int64_t)i, ssize, inner);
    i += 1.0;
  }
  int rc = overflow_verdict(n, t, ovf_at);
  for (int64_t v = 0; v < n; ++v) store_dist(kind, dist_out, v, t[v]);
  free(t); free(treq); free(tb); free(S); free(ovf_at);
  return rc;
}

/*
 * Meyer-Sanders delta-stepping with explicit buckets (Sec. III; Fig. 1 right):
 *   relax(v, x): if x < tent(v): move v from B[floor(tent(v)/delta)] to
 *                B[floor(x/delta)]; tent(v) = x
 *   tent = inf; relax(s, 0); i = 0
 *   while B is not empty:
 *     S = {}
 *     while B[i] is not empty:
 *       Req = {(w, tent(v) + c(v,w)) : v in B[i], (v,w) light}
 *       S = S u B[i]; B[i] = {}
 *       for (v, x) in Req: relax(v, x)
 *     Req = {(w, tent(v) + c(v,w)) : v in S, (v,w) heavy}
 *     for (v, x) in Req: relax(v, x)
 *     i = i + 1
 * Bucket membership is kept as one bucket index per vertex (-1 = in no bucket).
 */
typedef struct { int64_t v; double x; } request;

static void relax_set(int64_t v, double x, double *tent, int64_t *bidx, double dl) {
  if (x < tent[v]) {
    bidx[v] = bucket_of(x, dl);
    tent[v] = x;
  }
}

int orc_delta_sets(int64_t n, const int64_t *rp, const int32_t *col, const void *w, int kind, double delta,
                   int32_t src, void *dist_out, orc_trace *tr) {
  if (!check_args(n, rp, col, src) || kind < 0 || kind > 2 || !(delta > 0) || isinf(delta)) return ORC_BADARG;
  double dl = split_threshold(kind, delta);
  int64_t m = rp[n];
  double *tent = malloc(sizeof(double) * n);
  int64_t *bidx = malloc(sizeof(int64_t) * n);
  unsigned char *S = malloc(n), *ovf_at = calloc(n, 1);
  request *req = malloc(sizeof(request) * (m + 1));
  int64_t *members = malloc(sizeof(int64_t) * n);
  if (!tent || !bidx || !S || !ovf_at || !req || !members) {
    free(tent); free(bidx); free(S); free(ovf_at); free(req); free(members); return ORC_NOMEM;
  }
  if (tr) {
    tr->nbuckets = tr->outer_iters = tr->light_relax = tr->heavy_relax = tr->late_requests = 0;
    tr->s_conflicts = 0;
    if (tr->s_bucket) for (int64_t v = 0; v < n; ++v) tr->s_bucket[v] = -1;
  }
  for (int64_t v = 0; v < n; ++v) { tent[v] = INFINITY; bidx[v] = -1; }
  relax_set(src, 0.0, tent, bidx, dl);
  int64_t i = 0;
  int rc = ORC_OK;
  for (;;) {
    int64_t lowest = -1;
    for (int64_t v = 0; v < n; ++v)
      if (bidx[v] >= 0 && (lowest < 0 || bidx[v] < lowest)) lowest = bidx[v];
    if (lowest < 0) break;           /* B is empty */
    if (lowest < i) { rc = ORC_CLOSED_BUCKET; break; }
    if (tr) tr->outer_iters++;
    memset(S, 0, n);
    int64_t inner = 0;
    for (;;) {
      int64_t nb = 0;
      for (int64_t v = 0; v < n; ++v)
        if (bidx[v] == i) members[nb++] = v;
      if (nb == 0) break;
      inner++;
      int64_t nreq = 0;
      for (int64_t k = 0; k < nb; ++k) {
        int64_t u = members[k];
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
          double we = weight_of(kind, w, e);
          if (!is_light(we, dl)) continue;
          if (tr) tr->light_relax++;
          int ovf;
          double c = plus(kind, tent[u], we, &ovf);
          if (ovf) { ovf_at[col[e]] = 1; continue; }
          req[nreq].v = col[e]; req[nreq].x = c; nreq++;
        }
      }
      for (int64_t k = 0; k < nb; ++k) {
        S[members[k]] = 1;
        bidx[members[k]] = -1;
        trace_s_member(tr, members[k], i);
      }
      for (int64_t k = 0; k < nreq; ++k) relax_set(req[k].v, req[k].x, tent, bidx, dl);
    }
    int64_t nreq = 0, ssize = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (!S[u]) continue;
      ssize++;
      for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
        double we = weight_of(kind, w, e);
        if (!is_heavy(we, dl)) continue;
        if (tr) tr->heavy_relax++;
        int ovf;
        double c = plus(kind, tent[u], we, &ovf);
        if (ovf) { ovf_at[col[e]] = 1; continue; }
        req[nreq].v = col[e]; req[nreq].x = c; nreq++;
      }
    }
    for (int64_t k = 0; k < nreq; ++k) {
      if (tr && req[k].x < tent[req[k].v] && lt_multiple(req[k].x, (double)(i + 1), dl)) tr->late_requests++;
      relax_set(req[k].v, req[k].x, tent, bidx, dl);
    }
    trace_bucket(tr, i, ssize, inner);
    i += 1;
  }
  if (rc == ORC_OK) rc = overflow_verdict(n, tent, ovf_at);
  for (int64_t v = 0; v < n; ++v) store_dist(kind, dist_out, v, tent[v]);
  free(tent); free(bidx); free(S); free(ovf_at); free(req); free(members);
  return rc;
}

/* ------------------------------------------------------------ Bellman-Ford */

/* Brute force: rounds of relaxing every edge until nothing changes (at most n
 * rounds for positive weights). ORC_U32 sums are kept exact (no 2^32 cap) and
 * the overflow verdict is taken on the final values; reachability is tracked
 * separately so that an fp32 sum that rounds to +inf is told apart from "no path". */
int orc_bellman_ford(int64_t n, const int64_t *rp, const int32_t *col, const void *w, int kind, int32_t src,
                     void *dist_out) {
  if (!check_args(n, rp, col, src) || kind < 0 || kind > 2) return ORC_BADARG;
  double *d = malloc(sizeof(double) * n);
  unsigned char *reach = calloc(n, 1);
  if (!d || !reach) { free(d); free(reach); return ORC_NOMEM; }
  for (int64_t v = 0; v < n; ++v) d[v] = INFINITY;
  d[src] = 0.0;
  reach[src] = 1;
  for (int64_t round = 0; round <= n; ++round) {
    int changed = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (!reach[u]) continue;
      for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
        int64_t v = col[e];
        if (!reach[v]) { reach[v] = 1; changed = 1; }
        if (isinf(d[u])) continue;
        double we = weight_of(kind, w, e), c;
        if (kind == ORC_U32) c = d[u] + we; /* exact while below 2^53 */
        else if (kind == ORC_F32) c = (double)((float)d[u] + (float)we);
        else c = d[u] + we;
        if (c < d[v]) { d[v] = c; changed = 1; }
      }
    }
    if (!changed) break;
  }
  int rc = ORC_OK;
  for (int64_t v = 0; v < n; ++v) {
    if (!reach[v]) continue;
    if (isinf(d[v]) || (kind == ORC_U32 && d[v] > U32_MAX_DIST)) { rc = ORC_OVERFLOW; d[v] = INFINITY; }
  }
  for (int64_t v = 0; v < n; ++v) store_dist(kind, dist_out, v, d[v]);
  free(d); free(reach);
  return rc;
}

/* ------------------------------------------------------------ certificate */

/*
 * A candidate d is the shortest-path distance vector iff
 *   (a) d(s) = +0 and every entry is a value some path weight can take;
 *   (b) feasibility: for every edge (u,v,w) with d(u) finite, d(v) <= d(u) (+) w,
 *       and d(v) is finite whenever d(u) (+) w overflows is not representable;
 *   (c) every finite d(v) is reached from s through tight edges
 *       (d(u) finite and d(u) (+) w == d(v)).
 * (c) gives a path of weight d(v); (b) with the monotonicity of x -> x (+) w
 * gives d(v) <= weight of every path, by induction along the path; vertices with
 * d = inf then have no finite in-neighbour, so they are exactly the unreachable ones.
 */
int orc_certify(int64_t n, const int64_t *rp, const int32_t *col, const void *w, int kind, int32_t src,
                const void *dist) {
  if (!check_args(n, rp, col, src) || kind < 0 || kind > 2 || !dist) return -1;
  double *d = malloc(sizeof(double) * n);
  unsigned char *seen = calloc(n, 1);
  int64_t *queue = malloc(sizeof(int64_t) * n);
  if (!d || !seen || !queue) { free(d); free(seen); free(queue); return -1; }
  int verdict = CERT_OK;
  for (int64_t v = 0; v < n; ++v) d[v] = load_dist(kind, dist, v);
  for (int64_t v = 0; v < n && verdict == CERT_OK; ++v)
    if (isnan(d[v]) || d[v] < 0.0 || (d[v] == 0.0 && signbit(d[v]))) verdict = CERT_VALUE;
  if (verdict == CERT_OK && d[src] != 0.0) verdict = CERT_SOURCE;
  for (int64_t u = 0; u < n && verdict == CERT_OK; ++u) {
    if (isinf(d[u])) continue;
    for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
      int ovf;
      double c = plus(kind, d[u], weight_of(kind, w, e), &ovf);
      if (ovf) {
        if (isinf(d[col[e]])) { verdict = CERT_OVERFLOW; break; }
        continue;
      }
      if (c < d[col[e]]) { verdict = CERT_FEASIBLE; break; }
    }
  }
  if (verdict == CERT_OK) {
    int64_t head = 0, tail = 0;
    queue[tail++] = src;
    seen[src] = 1;
    while (head < tail) {
      int64_t u = queue[head++];
      for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
        int64_t v = col[e];
        if (seen[v]) continue;
        int ovf;
        double c = plus(kind, d[u], weight_of(kind, w, e), &ovf);
        if (!ovf && c == d[v]) { seen[v] = 1; queue[tail++] = v; }
      }
    }
    for (int64_t v = 0; v < n; ++v)
      if (!isinf(d[v]) && !seen[v]) { verdict = CERT_TIGHT; break; }
  }
  free(d); free(seen); free(queue);
  return verdict;
}

/* ------------------------------------------------------------ adjoint */

/*
 * Gradient of L = sum over reached v of grad_dist[v] * d(v) with respect to
 * the edge weights, through the shortest-path tree (reverse accumulation).
 *   parent of v != s (d(v) finite): a tight in-edge (d(u) finite and
 *   d(u) (+) w == d(v)) from a strictly closer vertex (d(u) < d(v)), the one
 *   with the smallest edge index. In exact arithmetic every tight edge is of
 *   that kind. With rounding, d(u) (+) w can equal d(u) (absorption in
 *   binary32 / binary64), so a vertex may be tight only through in-edges from
 *   vertices at its own distance, and those edges can form cycles. Such
 *   vertices take their parent in rounds: round 0 holds s and every vertex
 *   with a strictly-closer parent; round k gives each still unresolved vertex
 *   the smallest-index tight in-edge from a vertex resolved in round k - 1.
 *   The parents then form a tree. d(v) is the fold of the weights along its
 *   tree path, so dd(v)/dw_e = 1 for the edges of that path and 0 otherwise,
 *   and dL/dw_e for e = (parent(v), v) is the sum of grad_dist over the
 *   subtree below v (grad_dist of s and of unreached vertices is ignored).
 *   Where several shortest paths tie, this is the gradient along the chosen
 *   tree (a subgradient).
 * grad_w is ACCUMULATED (+=), in double. parent_edge (optional) receives the
 * chosen edge index of every vertex, -1 for s and unreached vertices.
 * Returns ORC_BADARG when dist is not a shortest-path vector (a reached vertex
 * without a tight in-edge, or parent pointers that do not lead to s).
 */
int orc_sp_gradient(int64_t n, const int64_t *rp, const int32_t *col, const void *w, int kind, int32_t src,
                    const void *dist, const double *grad_dist, double *grad_w, int64_t *parent_edge) {
  if (!check_args(n, rp, col, src) || kind < 0 || kind > 2 || !dist || !grad_dist || !grad_w) return ORC_BADARG;
  double *d = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * n);
  int64_t *pe = malloc(sizeof(int64_t) * n), *pv = malloc(sizeof(int64_t) * n);
  int64_t *nchild = calloc(n + 1, sizeof(int64_t)), *child = malloc(sizeof(int64_t) * (n + 1));
  int64_t *stack = malloc(sizeof(int64_t) * (n + 1)), *order = malloc(sizeof(int64_t) * (n + 1));
  int64_t *round_of = malloc(sizeof(int64_t) * (n + 1));
  if (!d || !g || !pe || !pv || !nchild || !child || !stack || !order || !round_of) {
    free(d); free(g); free(pe); free(pv); free(nchild); free(child); free(stack); free(order); free(round_of);
    return ORC_NOMEM;
  }
  int rc = ORC_OK;
  for (int64_t v = 0; v < n; ++v) { d[v] = load_dist(kind, dist, v); pe[v] = -1; pv[v] = -1; }
  /* parents: smallest-index tight in-edge from a strictly closer vertex */
  for (int64_t u = 0; u < n; ++u) {
    if (isinf(d[u])) continue;
    for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
      int64_t v = col[e];
      if (v == src) continue;
      int ovf;
      double c = plus(kind, d[u], weight_of(kind, w, e), &ovf);
      if (!ovf && c == d[v] && d[u] < d[v] && (pe[v] < 0 || e < pe[v])) { pe[v] = e; pv[v] = u; }
    }
  }
  /* vertices tight only through equal-distance in-edges: rounds from the resolved ones */
  for (int64_t v = 0; v < n; ++v) round_of[v] = (!isinf(d[v]) && (v == src || pe[v] >= 0)) ? 0 : -1;
  for (int64_t k = 1;; ++k) {
    int grew = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (round_of[u] != k - 1) continue;
      for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
        int64_t v = col[e];
        if (v == src || isinf(d[v]) || (round_of[v] >= 0 && round_of[v] < k)) continue;
        int ovf;
        double c = plus(kind, d[u], weight_of(kind, w, e), &ovf);
        if (ovf || c != d[v]) continue;
        if (round_of[v] < 0) { round_of[v] = k; pe[v] = e; pv[v] = u; grew = 1; }
        else if (e < pe[v]) { pe[v] = e; pv[v] = u; }
      }
    }
    if (!grew) break;
  }
  int64_t reached = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (isinf(d[v])) continue;
    reached++;
    if (v != src && pe[v] < 0) rc = ORC_BADARG;
  }
  if (rc == ORC_OK) {
    /* children lists (CSR over parent vertices) */
    for (int64_t v = 0; v < n; ++v) if (pv[v] >= 0) nchild[pv[v] + 1]++;
    for (int64_t v = 0; v < n; ++v) nchild[v + 1] += nchild[v];
    int64_t *fill = calloc(n, sizeof(int64_t));
    if (!fill) rc = ORC_NOMEM;
    else {
      for (int64_t v = 0; v < n; ++v) if (pv[v] >= 0) child[nchild[pv[v]] + fill[pv[v]]++] = v;
      free(fill);
      /* preorder from s; children come after their parent, so a reverse walk
       * visits every child before its parent */
      int64_t top = 0, len = 0;
      stack[top++] = src;
      while (top > 0) {
        int64_t v = stack[--top];
        order[len++] = v;
        for (int64_t k = nchild[v]; k < nchild[v + 1]; ++k) stack[top++] = child[k];
      }
      if (len != reached) rc = ORC_BADARG; /* parent pointers with a cycle */
      for (int64_t v = 0; v < n; ++v) g[v] = (isinf(d[v]) || v == src) ? 0.0 : grad_dist[v];
      for (int64_t k = len - 1; k >= 0 && rc == ORC_OK; --k) {
        int64_t v = order[k];
        if (v == src) continue;
        grad_w[pe[v]] += g[v];
        g[pv[v]] += g[v];
      }
    }
  }
  if (parent_edge) for (int64_t v = 0; v < n; ++v) parent_edge[v] = pe[v];
  free(d); free(g); free(pe); free(pv); free(nchild); free(child); free(stack); free(order); free(round_of);
  return rc;
}

/* ------------------------------------------------------------ many sources on host threads */

/*
 * Timing aid for the CPU baseline: orc_dijkstra for each of k sources (row r of
 * dist_out <- sources[r]), spread over `threads` POSIX threads, each taking the
 * next source from a shared counter. The arithmetic is orc_dijkstra's, unchanged.
 * Returns the first non-OK status of any row (ORC_OK if none).
 */
typedef struct {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  const void *w;
  int kind;
  const int32_t *sources;
  int32_t k;
  char *out;
  size_t row_bytes;
  int32_t next;
  int rc;
  pthread_mutex_t lock;
} many_job;

static void *many_worker(void *arg) {
  many_job *j = arg;
  for (;;) {
    pthread_mutex_lock(&j->lock);
    int32_t r = j->next++;
    pthread_mutex_unlock(&j->lock);
    if (r >= j->k) break;
    int rc = orc_dijkstra(j->n, j->rp, j->col, j->w, j->kind, j->sources[r], j->out + (size_t)r * j->row_bytes);
    if (rc != ORC_OK) {
      pthread_mutex_lock(&j->lock);
      if (j->rc == ORC_OK) j->rc = rc;
      pthread_mutex_unlock(&j->lock);
    }
  }
  return NULL;
}

int orc_dijkstra_many(int64_t n, const int64_t *rp, const int32_t *col, const void *w, int kind,
                      const int32_t *sources, int32_t k, void *dist_out, int32_t threads) {
  if (k < 0 || threads < 1 || !sources || !dist_out || kind < 0 || kind > 2) return ORC_BADARG;
  many_job j = {n, rp, col, w, kind, sources, k, dist_out, (size_t)n * (kind == ORC_F64 ? 8 : 4), 0, ORC_OK,
                PTHREAD_MUTEX_INITIALIZER};
  if (threads > k) threads = k > 0 ? k : 1;
  pthread_t *tid = malloc(sizeof(pthread_t) * threads);
  if (!tid) return ORC_NOMEM;
  int started = 0;
  for (int t = 0; t < threads; ++t)
    if (pthread_create(&tid[t], NULL, many_worker, &j) == 0) ++started;
  if (started == 0) many_worker(&j);
  for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
  free(tid);
  return j.rc;
}
