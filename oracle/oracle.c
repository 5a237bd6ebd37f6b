/*
 * CPU oracle for exact triangle counting (Arifuzzaman, Khan and Marathe,
 * "Distributed-Memory Parallel Algorithms for Counting and Listing Triangles
 * in Big Graphs", arXiv 1706.05151).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library may include, link or
 * call this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it. It shares no code, header or constant table with
 * the GPU path.
 *
 * Two independent routes are provided:
 *   (1) Definitions (Section 2, Preliminaries): T_v is the number of edges among
 *       the neighbours of v; T = (sum_v T_v)/3; C_v = T_v / C(d_v,2). Computed
 *       from the full sorted adjacency by set intersection, with no node order.
 *   (2) NodeIteratorN (Section 3, the algorithm figure after Eq. (1)): orient
 *       each edge by the degree order of Eq. (1), sort each N_v ascending, and
 *       add |N_v ∩ N_u| for every v and u in N_v; per-node counts follow the
 *       local-count figure of Section 9 and listing the figure of Section 8.
 * The sparsified count (Section 7) keeps each undirected edge independently;
 * the keep decision is a SplitMix64 hash (Steele, Lea and Flood, 2014) of the
 * seed and the edge, compared with q scaled to 2^64.
 *
 * Everything is serial and unoptimised except orc_count_nin_total_omp, which
 * only splits the outer loop of route (2) across threads for the largest
 * reference totals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------ helpers --- */

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* |A ∩ B| of two ascending arrays by a two-pointer merge */
static int64_t merge_count(const int32_t* a, int64_t na, const int32_t* b, int64_t nb) {
  int64_t i = 0, j = 0, c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) i++;
    else if (a[i] > b[j]) j++;
    else { c++; i++; j++; }
  }
  return c;
}

/* ----------------------------------------------------- the simple graph --- */

/*
 * The simple undirected graph of Section 2 from a raw edge list: ids must lie
 * in [0,n); self-loops are dropped; (u,v) and (v,u) and repeats are one edge.
 * Writes the m unique edges as lo[i] < hi[i], sorted by (lo,hi). lo/hi need
 * room for E entries. Returns m, or -1 if an id is out of range.
 */
int64_t orc_simple(const int32_t* src, const int32_t* dst, int64_t E, int32_t n,
                   int32_t* lo, int32_t* hi) {
  uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(E > 0 ? E : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < E; i++) {
    int32_t a = src[i], b = dst[i];
    if (a < 0 || a >= n || b < 0 || b >= n) { free(key); return -1; }
    if (a == b) continue;
    if (a > b) { int32_t t = a; a = b; b = t; }
    key[k++] = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
  }
  qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
  int64_t m = 0;
  for (int64_t i = 0; i < k; i++) {
    if (i > 0 && key[i] == key[i - 1]) continue;
    lo[m] = (int32_t)(key[i] >> 32);
    hi[m] = (int32_t)(key[i] & 0xffffffffu);
    m++;
  }
  free(key);
  return m;
}

/* d_v = |N(v)| (Section 2) */
void orc_degrees(const int32_t* lo, const int32_t* hi, int64_t m, int32_t n, int64_t* deg) {
  memset(deg, 0, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; i++) { deg[lo[i]]++; deg[hi[i]]++; }
}

/* Full adjacency: off[n+1], nbr[2m], each row ascending. */
void orc_full_adjacency(const int32_t* lo, const int32_t* hi, int64_t m, int32_t n,
                        int64_t* off, int32_t* nbr) {
  memset(off, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t i = 0; i < m; i++) { off[lo[i] + 1]++; off[hi[i] + 1]++; }
  for (int32_t v = 0; v < n; v++) off[v + 1] += off[v];
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  memcpy(pos, off, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; i++) {
    nbr[pos[lo[i]]++] = hi[i];
    nbr[pos[hi[i]]++] = lo[i];
  }
  for (int32_t v = 0; v < n; v++)
    qsort(nbr + off[v], (size_t)(off[v + 1] - off[v]), sizeof(int32_t), cmp_i32);
  free(pos);
}

/*
 * Coreness (the k-core order of Section 4, "An Optimal Node Ordering"): the
 * k-core is the largest subgraph in which every vertex has degree >= k, and
 * the coreness of v is the largest k whose k-core contains v. Computed by
 * peeling in degree buckets (Batagelj and Zaversnik, 2003): repeatedly remove
 * a vertex of smallest remaining degree; its remaining degree at removal,
 * raised to the running maximum, is its coreness. off/nbr: full adjacency.
 */
void orc_coreness(const int64_t* off, const int32_t* nbr, int32_t n, int32_t* core) {
  if (n <= 0) return;
  int32_t maxd = 0;
  int32_t* d = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; v++) {
    d[v] = (int32_t)(off[v + 1] - off[v]);
    if (d[v] > maxd) maxd = d[v];
  }
  /* bin[k] = first position of degree k in vert[]; vert sorted by degree; pos = inverse */
  int32_t* bin = (int32_t*)calloc((size_t)maxd + 2, sizeof(int32_t));
  int32_t* vert = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; v++) bin[d[v]]++;
  int32_t start = 0;
  for (int32_t k = 0; k <= maxd; k++) {
    int32_t c = bin[k];
    bin[k] = start;
    start += c;
  }
  for (int32_t v = 0; v < n; v++) {
    pos[v] = bin[d[v]];
    vert[pos[v]] = v;
    bin[d[v]]++;
  }
  for (int32_t k = maxd; k > 0; k--) bin[k] = bin[k - 1];
  bin[0] = 0;
  for (int32_t i = 0; i < n; i++) {
    int32_t v = vert[i];
    core[v] = d[v];
    for (int64_t j = off[v]; j < off[v + 1]; j++) {
      int32_t u = nbr[j];
      if (d[u] > d[v]) {
        /* move u to the front of its degree bucket, then shrink the bucket */
        int32_t du = d[u], pu = pos[u], pw = bin[du], w = vert[pw];
        if (u != w) {
          pos[u] = pw; vert[pw] = u;
          pos[w] = pu; vert[pu] = w;
        }
        bin[du]++;
        d[u]--;
      }
    }
  }
  free(d); free(bin); free(vert); free(pos);
}

/*
 * Load-balancing schemes of Section 5 (the cost-function table) and the cost
 * of the space-efficient algorithm of Section 6: f(v) for each vertex from the
 * oriented lists (rows by id, d^_v = |N_v|), the prefix F(t) = sum_{v<=t} f(v),
 * and the boundary nodes x_j = argmin_v F(v) >= j*alpha with alpha = F(n-1)/p
 * (compared exactly as F(v)*p >= j*F(n-1)); partition j holds the core nodes
 * [x_j, x_{j+1}). work[j] = sum over its core nodes v of the NodeIteratorN
 * merge cost sum_{u in N_v} (d^_v + d^_u) (Theorem 2).
 * scheme: 0 f=1, 1 f=d_v, 2 f=d^_v, 3 f=d_v*d^_v, 4 f=d^_v^2,
 *         5 f=sum_{u in N_v}(d^_v+d^_u), 6 f=sum_{u in Nfull_v - N_v}(d^_v+d^_u).
 */
void orc_partition_work(const int64_t* off, const int32_t* adj, const int64_t* deg, int32_t n, int scheme,
                        int32_t parts, int64_t* bounds, uint64_t* work) {
  uint64_t* f = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  uint64_t* cost = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  uint64_t* insum = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  for (int32_t u = 0; u < n; u++) {
    uint64_t du = (uint64_t)(off[u + 1] - off[u]);
    for (int64_t j = off[u]; j < off[u + 1]; j++) {
      int32_t v = adj[j];
      uint64_t dv = (uint64_t)(off[v + 1] - off[v]);
      cost[u] += du + dv;   /* u's merge against N_v */
      insum[v] += dv + du;  /* u is an in-neighbour of v */
    }
  }
  for (int32_t v = 0; v < n; v++) {
    uint64_t d = (uint64_t)deg[v], dh = (uint64_t)(off[v + 1] - off[v]);
    switch (scheme) {
      case 0: f[v] = 1; break;
      case 1: f[v] = d; break;
      case 2: f[v] = dh; break;
      case 3: f[v] = d * dh; break;
      case 4: f[v] = dh * dh; break;
      case 5: f[v] = cost[v]; break;
      default: f[v] = insum[v]; break;
    }
  }
  uint64_t total = 0;
  for (int32_t v = 0; v < n; v++) total += f[v];
  bounds[0] = 0;
  bounds[parts] = n;
  for (int32_t j = 1; j < parts; j++) {
    /* first v with F(v) * parts >= j * total */
    uint64_t F = 0;
    int32_t x = n;
    for (int32_t v = 0; v < n; v++) {
      F += f[v];
      if ((unsigned __int128)F * (unsigned)parts >= (unsigned __int128)total * (unsigned)j) { x = v; break; }
    }
    bounds[j] = x;
  }
  for (int32_t j = 0; j < parts; j++) {
    uint64_t w = 0;
    for (int64_t v = bounds[j]; v < bounds[j + 1]; v++) w += cost[v];
    work[j] = w;
  }
  free(f); free(cost); free(insum);
}

/* ----------------------------------------------- route (1): definitions --- */

/*
 * T_v = |{(u,w) in E : u,w in N(v)}| (Section 2). Each edge (u,w) among the
 * neighbours of v is seen from both u and w when summing |N(v) ∩ N(u)| over
 * u in N(v), hence the halving. Returns T = sum_v T_v / 3.
 */
uint64_t orc_local_counts_def(const int64_t* off, const int32_t* nbr, int32_t n, uint64_t* t) {
  uint64_t sum = 0;
  for (int32_t v = 0; v < n; v++) {
    uint64_t twice = 0;
    for (int64_t i = off[v]; i < off[v + 1]; i++) {
      int32_t u = nbr[i];
      twice += (uint64_t)merge_count(nbr + off[v], off[v + 1] - off[v], nbr + off[u], off[u + 1] - off[u]);
    }
    t[v] = twice / 2;
    sum += t[v];
  }
  return sum / 3;
}

/* ------------------------------------------------ route (2): NodeIteratorN --- */

/* u precedes v in the degree order of Eq. (1): d_u < d_v, ties by smaller id. */
static int precedes(const int64_t* deg, int32_t u, int32_t v) {
  return deg[u] < deg[v] || (deg[u] == deg[v] && u < v);
}

/*
 * Preprocessing of NodeIteratorN: for each edge (u,v), store v in N_u if
 * u precedes v, else u in N_v; then sort every N_v ascending (by id).
 * off[n+1], adj[m].
 */
void orc_orient(const int32_t* lo, const int32_t* hi, int64_t m, const int64_t* deg,
                int32_t n, int64_t* off, int32_t* adj) {
  memset(off, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t i = 0; i < m; i++) {
    int32_t a = lo[i], b = hi[i];
    int32_t s = precedes(deg, a, b) ? a : b;
    off[s + 1]++;
  }
  for (int32_t v = 0; v < n; v++) off[v + 1] += off[v];
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  memcpy(pos, off, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; i++) {
    int32_t a = lo[i], b = hi[i];
    if (precedes(deg, a, b)) adj[pos[a]++] = b;
    else adj[pos[b]++] = a;
  }
  for (int32_t v = 0; v < n; v++)
    qsort(adj + off[v], (size_t)(off[v + 1] - off[v]), sizeof(int32_t), cmp_i32);
  free(pos);
}

/*
 * Orientation by an arbitrary total order given as a key per vertex (ties by
 * id), used to check that any order counts each triangle once (Theorem 1) and
 * that the degree order minimises sum_v d_v * dhat_v (Theorem 3).
 */
void orc_orient_by_key(const int32_t* lo, const int32_t* hi, int64_t m, const int64_t* key,
                       int32_t n, int64_t* off, int32_t* adj) {
  orc_orient(lo, hi, m, key, n, off, adj);
}

/*
 * The counting loop of NodeIteratorN: for v in V, for u in N_v, S = N_v ∩ N_u,
 * T += |S|. With t != NULL each triangle (v,u,w) adds one to t_v, t_u and t_w
 * (local-count figure, Section 9). With tri != NULL the triangle is written as
 * its three ids in ascending order (listing figure, Section 8), at most cap of
 * them. Returns T.
 */
uint64_t orc_count_nin(const int64_t* off, const int32_t* adj, int32_t n, uint64_t* t,
                       int32_t* tri, int64_t cap) {
  uint64_t T = 0;
  if (t) memset(t, 0, sizeof(uint64_t) * (size_t)n);
  for (int32_t v = 0; v < n; v++) {
    const int32_t* nv = adj + off[v];
    int64_t dv = off[v + 1] - off[v];
    for (int64_t k = 0; k < dv; k++) {
      int32_t u = nv[k];
      const int32_t* nu = adj + off[u];
      int64_t du = off[u + 1] - off[u];
      int64_t i = 0, j = 0;
      while (i < dv && j < du) {
        if (nv[i] < nu[j]) i++;
        else if (nv[i] > nu[j]) j++;
        else {
          int32_t w = nv[i];
          if (t) { t[v]++; t[u]++; t[w]++; }
          if (tri && (int64_t)T < cap) {
            int32_t a = v, b = u, c = w, x;
            if (a > b) { x = a; a = b; b = x; }
            if (b > c) { x = b; b = c; c = x; }
            if (a > b) { x = a; a = b; b = x; }
            tri[3 * T + 0] = a;
            tri[3 * T + 1] = b;
            tri[3 * T + 2] = c;
          }
          T++;
          i++;
          j++;
        }
      }
    }
  }
  return T;
}

/* T only, outer loop over v split across threads (results equal orc_count_nin). */
uint64_t orc_count_nin_total_omp(const int64_t* off, const int32_t* adj, int32_t n) {
  uint64_t T = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : T)
  for (int32_t v = 0; v < n; v++) {
    for (int64_t k = off[v]; k < off[v + 1]; k++) {
      int32_t u = adj[k];
      T += (uint64_t)merge_count(adj + off[v], off[v + 1] - off[v], adj + off[u], off[u + 1] - off[u]);
    }
  }
  return T;
}

/* ------------------------------------------------------------- shards --- */

static const int64_t* g_pos_key; /* key of the qsort below (single-threaded use) */
static int cmp_by_key_then_id(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  if (g_pos_key[x] != g_pos_key[y]) return g_pos_key[x] < g_pos_key[y] ? -1 : 1;
  return (x > y) - (x < y);
}

/*
 * Positions in a total order given by a key per vertex, ties by smaller id
 * (Eq. (1) when the key is the degree): pos[v] = number of vertices that
 * precede v.
 */
void orc_order_positions(const int64_t* key, int32_t n, int32_t* pos) {
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t v = 0; v < n; v++) ids[v] = v;
  g_pos_key = key;
  qsort(ids, (size_t)n, sizeof(int32_t), cmp_by_key_then_id);
  for (int32_t r = 0; r < n; r++) pos[ids[r]] = r;
  free(ids);
}

/*
 * Core-node shards over positions (the overlapping partitions of Section 5
 * with the partitioning done on the orientation order). The cost at position
 * pos[v] is, for cost 0, sum_{u in N_v} (dhat_v + dhat_u) (the DPD row of the
 * cost-function table) and, for cost 1, 2 dhat_v (dhat_v - 1) + 16 dhat_v +
 * sum_{u in N_v} dhat_u (four times the C(dhat_v,2) wedges of v plus 4 per
 * oriented edge, and a quarter of the lengths of the lists N_u). F is its
 * inclusive prefix over positions, and bounds[j] (0 < j < k) the first
 * position p with F(p)*k >= j*F(n-1) (the boundary rule x_j = argmin F >=
 * j*alpha, exactly); bounds[0] = 0, bounds[k] = n.
 */
void orc_shard_bounds(const int64_t* off, const int32_t* adj, int32_t n, const int32_t* pos, int32_t k, int cost,
                      int64_t* bounds) {
  uint64_t* f = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  for (int32_t v = 0; v < n; v++) {
    uint64_t dv = (uint64_t)(off[v + 1] - off[v]), x = 0;
    for (int64_t j = off[v]; j < off[v + 1]; j++) {
      int32_t u = adj[j];
      x += (cost == 0 ? dv : 0) + (uint64_t)(off[u + 1] - off[u]);
    }
    if (cost == 1) x += 2 * dv * (dv > 0 ? dv - 1 : 0) + 16 * dv;
    f[pos[v]] = x;
  }
  uint64_t total = 0;
  for (int32_t p = 0; p < n; p++) total += f[p];
  bounds[0] = 0;
  bounds[k] = n;
  for (int32_t j = 1; j < k; j++) {
    uint64_t F = 0;
    int32_t x = n;
    for (int32_t p = 0; p < n; p++) {
      F += f[p];
      if ((unsigned __int128)F * (unsigned)k >= (unsigned __int128)total * (unsigned)j) { x = p; break; }
    }
    bounds[j] = x;
  }
  free(f);
}

/*
 * The counting loop of NodeIteratorN over the core nodes v whose position
 * lies in [p0, p1): each triangle is counted once, at its lowest vertex.
 */
uint64_t orc_count_nin_pos_range(const int64_t* off, const int32_t* adj, int32_t n, const int32_t* pos,
                                 int32_t p0, int32_t p1) {
  uint64_t T = 0;
  for (int32_t v = 0; v < n; v++) {
    if (pos[v] < p0 || pos[v] >= p1) continue;
    for (int64_t k = off[v]; k < off[v + 1]; k++) {
      int32_t u = adj[k];
      T += (uint64_t)merge_count(adj + off[v], off[v + 1] - off[v], adj + off[u], off[u + 1] - off[u]);
    }
  }
  return T;
}

/* Merge work of Theorem 2: W = sum over oriented edges (v,u) of (dhat_v + dhat_u). */
uint64_t orc_work(const int64_t* off, const int32_t* adj, int32_t n) {
  uint64_t W = 0;
  for (int32_t v = 0; v < n; v++)
    for (int64_t k = off[v]; k < off[v + 1]; k++) {
      int32_t u = adj[k];
      W += (uint64_t)((off[v + 1] - off[v]) + (off[u + 1] - off[u]));
    }
  return W;
}

/* NodeIterator++ (Section 3, first algorithm figure): for v, for u in N(v) with
 * v before u, for w in N(v) with u before w, test (u,w) in E by binary search
 * in the full sorted adjacency of u. Independent of the oriented lists. */
uint64_t orc_count_nodeiterpp(const int64_t* off, const int32_t* nbr, const int64_t* deg, int32_t n) {
  uint64_t T = 0;
  for (int32_t v = 0; v < n; v++)
    for (int64_t i = off[v]; i < off[v + 1]; i++) {
      int32_t u = nbr[i];
      if (!precedes(deg, v, u)) continue;
      for (int64_t j = off[v]; j < off[v + 1]; j++) {
        int32_t w = nbr[j];
        if (!precedes(deg, u, w)) continue;
        int32_t key = w;
        if (bsearch(&key, nbr + off[u], (size_t)(off[u + 1] - off[u]), sizeof(int32_t), cmp_i32)) T++;
      }
    }
  return T;
}

/* ------------------------------------------------------------ outputs --- */

static int cmp_tri(const void* a, const void* b) {
  const int32_t* x = (const int32_t*)a;
  const int32_t* y = (const int32_t*)b;
  for (int i = 0; i < 3; i++)
    if (x[i] != y[i]) return (x[i] > y[i]) - (x[i] < y[i]);
  return 0;
}

/* Sort a list of T triangles (each ascending) lexicographically. */
void orc_sort_triples(int32_t* tri, int64_t T) {
  qsort(tri, (size_t)T, 3 * sizeof(int32_t), cmp_tri);
}

/* C_v = T_v / C(d_v,2) (Section 2): numerator, denominator and the double
 * quotient; nodes with d_v < 2 get 0/0 and C_v = 0. */
void orc_clustering(const uint64_t* t, const int64_t* deg, int32_t n, uint64_t* num,
                    uint64_t* den, double* c) {
  for (int32_t v = 0; v < n; v++) {
    uint64_t d = (uint64_t)deg[v];
    num[v] = t[v];
    den[v] = d >= 2 ? d * (d - 1) / 2 : 0;
    c[v] = den[v] ? (double)num[v] / (double)den[v] : 0.0;
  }
}

/* ------------------------------------------------------- sparsification --- */

static uint64_t orc_splitmix64_finalizer(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Domain constant separating the sampler's stream from any other use of the seed. */
#define ORC_SPARSIFY_DOMAIN 0x5350415253494659ULL

/* Keep threshold: q scaled to 2^64 (q in (0,1)); q >= 1 keeps every edge. */
uint64_t orc_keep_threshold(double q) {
  if (q >= 1.0) return UINT64_MAX;
  return (uint64_t)ldexp(q, 64);
}

/* 1 if undirected edge {a,b} (a < b) is retained under (q, seed). */
int orc_keep(int32_t a, int32_t b, double q, uint64_t seed) {
  if (q >= 1.0) return 1;
  uint64_t h = orc_splitmix64_finalizer(orc_splitmix64_finalizer(seed ^ ORC_SPARSIFY_DOMAIN) ^
                                        (((uint64_t)(uint32_t)a << 32) | (uint32_t)b));
  return h < orc_keep_threshold(q);
}

/*
 * Seed of shard i's independent sample: output i+1 of the SplitMix64
 * generator (Steele, Lea and Flood, 2014) started at `seed`, i.e. the
 * finaliser applied to seed + (i+1) * 0x9E3779B97F4A7C15.
 */
uint64_t orc_partition_seed(uint64_t seed, int32_t i) {
  return orc_splitmix64_finalizer(seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL);
}

/* Retained subset of the unique edges lo<hi; returns m'. */
int64_t orc_sparsify(const int32_t* lo, const int32_t* hi, int64_t m, double q, uint64_t seed,
                     int32_t* klo, int32_t* khi) {
  int64_t k = 0;
  for (int64_t i = 0; i < m; i++)
    if (orc_keep(lo[i], hi[i], q, seed)) { klo[k] = lo[i]; khi[k] = hi[i]; k++; }
  return k;
}

/* The unbiased estimate T_s / q^3 (Section 7). */
double orc_estimate(uint64_t Ts, double q) { return (double)Ts / ((q * q) * q); }

/* -------------------------------------------------- sampled definitions --- */

/*
 * T_v and d_v by the definition, for k <= 64 sampled vertices, straight from a
 * raw edge list (loops and duplicates allowed) without building the graph:
 * pass 1 collects each sample's neighbour set; pass 2 collects the distinct
 * edges whose both ends are neighbours of a sample. Used at sizes where the
 * whole-graph routes are too slow. Returns 0, or -1 on bad arguments.
 */
int orc_sampled_local(const int32_t* src, const int32_t* dst, int64_t E, int32_t n,
                      const int32_t* sample, int32_t k, uint64_t* t_out, int64_t* deg_out) {
  if (k < 0 || k > 64) return -1;
  uint64_t* is_sample = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
  for (int32_t s = 0; s < k; s++) is_sample[sample[s]] |= 1ULL << s;
  /* pass 1: neighbour lists */
  int64_t* cnt = (int64_t*)calloc((size_t)k, sizeof(int64_t));
  for (int64_t i = 0; i < E; i++) {
    int32_t a = src[i], b = dst[i];
    if (a == b) continue;
    uint64_t ma = is_sample[a], mb = is_sample[b];
    for (int32_t s = 0; s < k; s++) {
      if (ma >> s & 1) cnt[s]++;
      if (mb >> s & 1) cnt[s]++;
    }
  }
  int32_t** nb = (int32_t**)malloc(sizeof(int32_t*) * (size_t)(k > 0 ? k : 1));
  int64_t* len = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
  for (int32_t s = 0; s < k; s++) nb[s] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt[s] + 1));
  for (int64_t i = 0; i < E; i++) {
    int32_t a = src[i], b = dst[i];
    if (a == b) continue;
    uint64_t ma = is_sample[a], mb = is_sample[b];
    if (!(ma | mb)) continue;
    for (int32_t s = 0; s < k; s++) {
      if (ma >> s & 1) nb[s][len[s]++] = b;
      if (mb >> s & 1) nb[s][len[s]++] = a;
    }
  }
  uint64_t* in_nbhd = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
  for (int32_t s = 0; s < k; s++) {
    qsort(nb[s], (size_t)len[s], sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t i = 0; i < len[s]; i++)
      if (i == 0 || nb[s][i] != nb[s][i - 1]) nb[s][u++] = nb[s][i];
    len[s] = u;
    deg_out[s] = u;
    for (int64_t i = 0; i < u; i++) in_nbhd[nb[s][i]] |= 1ULL << s;
  }
  /* pass 2: edges among the neighbours */
  int64_t* ecnt = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
  for (int64_t i = 0; i < E; i++) {
    int32_t a = src[i], b = dst[i];
    if (a == b) continue;
    uint64_t mm = in_nbhd[a] & in_nbhd[b];
    for (int32_t s = 0; s < k; s++)
      if (mm >> s & 1) ecnt[s]++;
  }
  uint64_t** ek = (uint64_t**)malloc(sizeof(uint64_t*) * (size_t)(k > 0 ? k : 1));
  int64_t* elen = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
  for (int32_t s = 0; s < k; s++) ek[s] = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(ecnt[s] + 1));
  for (int64_t i = 0; i < E; i++) {
    int32_t a = src[i], b = dst[i];
    if (a == b) continue;
    uint64_t mm = in_nbhd[a] & in_nbhd[b];
    if (!mm) continue;
    if (a > b) { int32_t x = a; a = b; b = x; }
    uint64_t key = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
    for (int32_t s = 0; s < k; s++)
      if (mm >> s & 1) ek[s][elen[s]++] = key;
  }
  for (int32_t s = 0; s < k; s++) {
    qsort(ek[s], (size_t)elen[s], sizeof(uint64_t), cmp_u64);
    uint64_t u = 0;
    for (int64_t i = 0; i < elen[s]; i++)
      if (i == 0 || ek[s][i] != ek[s][i - 1]) u++;
    t_out[s] = u;
    free(ek[s]);
    free(nb[s]);
  }
  free(ek); free(elen); free(ecnt); free(in_nbhd); free(nb); free(len); free(cnt); free(is_sample);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
