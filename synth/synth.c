/*
 * Seeded synthetic graph generators: the inputs of every test and benchmark.
 *
 * This module holds no part of the triangle-counting method. It only draws
 * edge lists; both the CPU oracle and the GPU library consume its output.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: the value for counter c under stream key k is the (c+1)-th output
 * of a SplitMix64 sequence whose state starts at k. Every draw is therefore a
 * pure function of (seed, stream, counter), independent of thread count.
 *
 * Graph models (the paper's dataset table uses Gnp and PA networks, and
 * power-law real networks for which R-MAT stands in):
 *   - Erdos-Renyi G(n,q) over all pairs i<j, by geometric skipping per row
 *     (Batagelj and Brandes, Phys. Rev. E 71, 2005).
 *   - Preferential attachment (Barabasi-Albert): seed clique K_{k+1}, then each
 *     new node picks k distinct targets from the repeated-endpoint list.
 *   - R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004) with quadrant
 *     probabilities (a,b,c,d), no noise and no vertex permutation.
 * Raw outputs may contain self-loops and duplicate pairs (R-MAT does); the
 * consumers drop them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SM64_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* The ctr-th output of a SplitMix64 sequence started at state `key`. */
static inline uint64_t sm64_at(uint64_t key, uint64_t ctr) {
  return sm64_mix(key + (ctr + 1) * SM64_GAMMA);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return sm64_mix(sm64_mix(seed) ^ (stream * 0xd1b54a32d192ed03ULL + 0x632be59bd9b4e019ULL));
}

/* uniform double in [0,1) with 53 random bits */
static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, n) for n < 2^32 (multiply-high) */
static inline uint64_t below(uint64_t r, uint64_t n) { return ((r >> 32) * n) >> 32; }

uint64_t synth_splitmix_at(uint64_t key, uint64_t ctr) { return sm64_at(key, ctr); }
uint64_t synth_stream_key(uint64_t seed, uint64_t stream) { return stream_key(seed, stream); }

/* ------------------------------------------------------------------ ER --- */

/* Number of candidates skipped before the next kept pair: geometric(q). */
static inline int64_t geo_skip(double r, double lq) {
  /* floor(log(1-r)/log(1-q)) */
  double s = floor(log1p(-r) / lq);
  if (s > 4.0e18) s = 4.0e18;
  return (int64_t)s;
}

/*
 * Row i of G(n,q) holds the candidate pairs (i, j) for j in (i, n). Each row
 * uses its own stream so rows can be generated independently.
 * Pass 1 (dst == NULL) stores per-row counts in row_cnt; pass 2 writes edges
 * at the offsets in row_off.
 */
static void er_rows(int32_t n, double q, uint64_t seed, int64_t* row_cnt,
                    const int64_t* row_off, int32_t* src, int32_t* dst) {
  const double lq = log1p(-q);
  const uint64_t base = stream_key(seed, 0x4552);
#pragma omp parallel for schedule(dynamic, 256)
  for (int32_t i = 0; i < n - 1; i++) {
    uint64_t key = sm64_mix(base ^ ((uint64_t)i * SM64_GAMMA));
    uint64_t ctr = 0;
    int64_t j = (int64_t)i; /* last visited candidate */
    int64_t c = 0;
    int64_t w = row_off ? row_off[i] : 0;
    for (;;) {
      if (q >= 1.0) {
        j += 1;
      } else {
        double r = u01(sm64_at(key, ctr++));
        j += 1 + geo_skip(r, lq);
      }
      if (j >= n || j < 0) break;
      if (src) {
        src[w + c] = i;
        dst[w + c] = (int32_t)j;
      }
      c++;
    }
    if (row_cnt) row_cnt[i] = c;
  }
}

/* Returns the number of edges; writes them when src/dst are non-NULL
 * (call once with NULL to size the buffers). */
int64_t synth_er(int32_t n, double q, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 2 || !(q > 0.0)) return 0;
  int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  er_rows(n, q, seed, cnt, NULL, NULL, NULL);
  int64_t total = 0;
  for (int32_t i = 0; i < n; i++) {
    int64_t c = cnt[i];
    cnt[i] = total;
    total += c;
  }
  if (src && dst) er_rows(n, q, seed, NULL, cnt, src, dst);
  free(cnt);
  return total;
}

/* ------------------------------------------------------------------ BA --- */

/* Edge count of the model: C(k+1,2) for the seed clique plus k per new node. */
int64_t synth_ba_edges(int32_t n, int32_t k) {
  if (k < 1 || n <= k) return (int64_t)(n > 1 ? n : 0) * (n > 1 ? n - 1 : 0) / 2;
  return (int64_t)k * (k + 1) / 2 + (int64_t)(n - k - 1) * k;
}

int64_t synth_ba(int32_t n, int32_t k, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 2) return 0;
  if (k < 1) k = 1;
  int32_t s = (n <= k) ? n : k + 1; /* seed clique size */
  int64_t e = 0;
  int64_t total = synth_ba_edges(n, k);
  int32_t* ends = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * total + 2));
  int64_t nends = 0;
  for (int32_t a = 0; a < s; a++)
    for (int32_t b = a + 1; b < s; b++) {
      src[e] = b;
      dst[e] = a;
      e++;
      ends[nends++] = a;
      ends[nends++] = b;
    }
  const uint64_t key = stream_key(seed, 0x4241);
  uint64_t ctr = 0;
  int32_t* chosen = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t v = s; v < n; v++) {
    int32_t got = 0;
    while (got < k) {
      int32_t t = ends[below(sm64_at(key, ctr++), (uint64_t)nends)];
      int dup = 0;
      for (int32_t i = 0; i < got; i++)
        if (chosen[i] == t) { dup = 1; break; }
      if (!dup) chosen[got++] = t;
    }
    for (int32_t i = 0; i < k; i++) {
      src[e] = v;
      dst[e] = chosen[i];
      e++;
      ends[nends++] = v;
      ends[nends++] = chosen[i];
    }
  }
  free(chosen);
  free(ends);
  return e;
}

/* ---------------------------------------------------------------- RMAT --- */

/* E = num_edges draws of an R-MAT graph on 2^scale vertices. Each recursion
 * level consumes 32 random bits (two levels per 64-bit draw), compared with the
 * cumulative quadrant probabilities scaled to 2^32. */
void synth_rmat(int32_t scale, int64_t num_edges, double a, double b, double c,
                uint64_t seed, int32_t* src, int32_t* dst) {
  const double two32 = 4294967296.0;
  const uint64_t t1 = (uint64_t)(a * two32), t2 = (uint64_t)((a + b) * two32),
                 t3 = (uint64_t)((a + b + c) * two32);
  const uint64_t key = stream_key(seed, 0x524d);
  const uint64_t per_edge = (uint64_t)(scale + 1) / 2;
#pragma omp parallel for schedule(static, 65536)
  for (int64_t e = 0; e < num_edges; e++) {
    uint32_t s = 0, d = 0;
    const uint64_t c0 = (uint64_t)e * per_edge;
    uint64_t r = 0;
    for (int32_t l = 0; l < scale; l++) {
      uint64_t x;
      if ((l & 1) == 0) {
        r = sm64_at(key, c0 + (uint64_t)(l >> 1));
        x = r >> 32;
      } else {
        x = r & 0xffffffffULL;
      }
      uint32_t sb = (x >= t2), db = (x >= t1 && x < t2) || (x >= t3);
      s = (s << 1) | sb;
      d = (d << 1) | db;
    }
    src[e] = (int32_t)s;
    dst[e] = (int32_t)d;
  }
}

/* --------------------------------------------------------------- misc --- */

/* Draws `count` values of a stream: used for mixes (graph types, sizes, arrival
 * times) so every higher-level recipe shares the same counter-based source. */
void synth_draws(uint64_t seed, uint64_t stream, uint64_t first, int64_t count, uint64_t* out) {
  const uint64_t key = stream_key(seed, stream);
  for (int64_t i = 0; i < count; i++) out[i] = sm64_at(key, first + (uint64_t)i);
}

int synth_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
