/*
 * axsynth — seeded synthetic corpora and request traces (inputs only).
 *
 * Shapes follow the workloads the paper measures on (Setup; Table 2; the
 * self-overlap and depth statistics of the periodic-fill and memory-floor
 * sections): 16 KiB blocks, a median match near 7 B, roughly a quarter of
 * the bytes copied, short-period tandem repeats.  All constants not fixed by
 * the workload description are stated here.
 */
#include "axsynth.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- PRNG --- */

uint64_t axs_splitmix64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static double u01(uint64_t* s) { return (double)(axs_splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

/* Geometric on {1,2,...} with the given mean (> 1). */
static uint64_t geom(uint64_t* s, double mean) {
  double u = u01(s);
  double g = floor(log(1.0 - u) / log(1.0 - 1.0 / mean));
  if (g < 0) g = 0;
  if (g > 1e15) g = 1e15;
  return 1 + (uint64_t)g;
}

static double normal(uint64_t* s) {
  double u1 = 1.0 - u01(s); /* (0,1] */
  double u2 = u01(s);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static double lognormal(uint64_t* s, double mu, double sigma) { return exp(mu + sigma * normal(s)); }

/* Uniform integer in [a, b]. */
static uint64_t unif(uint64_t* s, uint64_t a, uint64_t b) {
  return a + (uint64_t)(u01(s) * (double)(b - a + 1));
}

/* ------------------------------------------------------------------ DNA --- */

static const uint8_t BASES[4] = {'A', 'C', 'G', 'T'};

typedef struct {
  double cum[64][4]; /* order-3 Markov rows (cumulative) */
  unsigned ctx;
} markov_t;

static void markov_init(markov_t* m, uint64_t* s) {
  for (int c = 0; c < 64; c++) {
    double g[4], t = 0;
    for (int k = 0; k < 4; k++) { /* Gamma(4,1) = -ln(u1 u2 u3 u4): Dirichlet(4,4,4,4) row */
      double p = 1.0;
      for (int j = 0; j < 4; j++) p *= (1.0 - u01(s));
      g[k] = -log(p);
      t += g[k];
    }
    double acc = 0;
    for (int k = 0; k < 4; k++) { acc += g[k] / t; m->cum[c][k] = acc; }
    m->cum[c][3] = 1.0;
  }
  m->ctx = (unsigned)unif(s, 0, 63);
}

static unsigned markov_next(markov_t* m, uint64_t* s) {
  double u = u01(s);
  const double* r = m->cum[m->ctx];
  unsigned b = u < r[0] ? 0 : u < r[1] ? 1 : u < r[2] ? 2 : 3;
  m->ctx = ((m->ctx << 2) | b) & 63;
  return b;
}

static unsigned base_code(uint8_t c) { return c == 'A' ? 0 : c == 'C' ? 1 : c == 'G' ? 2 : 3; }

int axs_dna(uint8_t* out, uint64_t n, uint64_t seed) {
  uint64_t s = seed * 0x2545F4914F6CDD1DULL + 0xD1B54A32D192ED03ULL;
  markov_t m;
  markov_init(&m, &s);
  uint64_t pos = 0;
  while (pos < n) {
    double u = u01(&s);
    if (u < 0.770) { /* Markov filler run */
      uint64_t len = geom(&s, 40.0);
      for (uint64_t k = 0; k < len && pos < n; k++) out[pos++] = BASES[markov_next(&m, &s)];
    } else if (u < 0.997) { /* planted copy of an earlier segment */
      uint64_t len;
      int longcopy = u01(&s) >= 0.99;
      if (!longcopy) {
        double l = floor(lognormal(&s, log(7.0), 0.75) + 0.5);
        len = l < 1 ? 1 : (uint64_t)l;
      } else {
        len = unif(&s, 200, 5000);
      }
      if (len > pos) len = pos;
      if (len == 0) continue;
      uint64_t src = unif(&s, 0, pos - len);
      for (uint64_t k = 0; k < len && pos < n; k++) {
        uint8_t b = out[src + k];
        if (longcopy && u01(&s) < 0.01) b = BASES[(base_code(b) + 1 + unif(&s, 0, 2)) & 3];
        out[pos++] = b;
        m.ctx = ((m.ctx << 2) | base_code(b)) & 63;
      }
    } else { /* tandem repeat: period 1..6 repeated 10..200 times */
      unsigned period = (unsigned)unif(&s, 1, 6);
      uint64_t reps = unif(&s, 10, 200);
      uint8_t unit[6];
      for (unsigned k = 0; k < period; k++) unit[k] = BASES[markov_next(&m, &s)];
      for (uint64_t r = 0; r < reps; r++)
        for (unsigned k = 0; k < period && pos < n; k++) out[pos++] = unit[k];
    }
  }
  /* lowercase: alternating runs, upper Geometric(700), lower Geometric(300) */
  pos = 0;
  while (pos < n) {
    pos += geom(&s, 700.0);
    uint64_t l = geom(&s, 300.0);
    for (uint64_t k = 0; k < l && pos < n; k++, pos++) out[pos] = (uint8_t)(out[pos] | 0x20);
  }
  /* N runs: alternating gap Geometric(202752) and run Geometric(2048) */
  pos = 0;
  while (pos < n) {
    pos += geom(&s, 202752.0);
    uint64_t l = geom(&s, 2048.0);
    for (uint64_t k = 0; k < l && pos < n; k++, pos++) out[pos] = 'N';
  }
  return 0;
}

/* ----------------------------------------------------------------- text --- */

#define VOCAB 50000

typedef struct {
  char w[VOCAB][13];
  uint8_t len[VOCAB];
  double cum[VOCAB]; /* Zipf(1.1) cumulative weights over ranks 1..VOCAB */
} vocab_t;

static uint64_t str_hash(const char* p, unsigned n) {
  uint64_t h = 1469598103934665603ULL;
  for (unsigned i = 0; i < n; i++) h = (h ^ (uint8_t)p[i]) * 1099511628211ULL;
  return h;
}

static int vocab_build(vocab_t* v, uint64_t* s) {
  const uint64_t cap = 1u << 17;
  int32_t* set = (int32_t*)malloc(cap * sizeof(int32_t));
  if (!set) return -1;
  for (uint64_t i = 0; i < cap; i++) set[i] = -1;
  int k = 0;
  while (k < VOCAB) {
    unsigned n = (unsigned)unif(s, 2, 12);
    char w[13];
    for (unsigned i = 0; i < n; i++) w[i] = (char)('a' + unif(s, 0, 25));
    uint64_t h = str_hash(w, n) & (cap - 1);
    int dup = 0;
    while (set[h] >= 0) {
      if (v->len[set[h]] == n && memcmp(v->w[set[h]], w, n) == 0) { dup = 1; break; }
      h = (h + 1) & (cap - 1);
    }
    if (dup) continue;
    set[h] = k;
    memcpy(v->w[k], w, n);
    v->len[k] = (uint8_t)n;
    k++;
  }
  free(set);
  double acc = 0;
  for (int r = 0; r < VOCAB; r++) { acc += pow((double)(r + 1), -1.1); v->cum[r] = acc; }
  for (int r = 0; r < VOCAB; r++) v->cum[r] /= acc;
  return 0;
}

static int zipf_word(const vocab_t* v, uint64_t* s) {
  double u = u01(s);
  int lo = 0, hi = VOCAB - 1;
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    if (v->cum[mid] < u) lo = mid + 1; else hi = mid;
  }
  return lo;
}

typedef struct {
  uint8_t* out;
  uint64_t n, pos, col, width;
} tw_t;

static void tw_put(tw_t* t, uint8_t c) {
  if (t->pos < t->n) t->out[t->pos++] = c;
  t->col = (c == '\n') ? 0 : t->col + 1;
}

/* A word boundary: newline when the line is past its drawn width, else space. */
static void tw_sep(tw_t* t, uint64_t* s) {
  if (t->col >= t->width) { tw_put(t, '\n'); t->width = unif(s, 72, 88); }
  else tw_put(t, ' ');
}

int axs_text(uint8_t* out, uint64_t n, uint64_t seed) {
  uint64_t s = seed * 0x2545F4914F6CDD1DULL + 0x9E3779B97F4A7C15ULL;
  vocab_t* v = (vocab_t*)malloc(sizeof(vocab_t));
  if (!v) return -1;
  if (vocab_build(v, &s)) { free(v); return -1; }
  uint64_t cap = 1024, ns = 0;
  uint64_t* st = (uint64_t*)malloc(cap * sizeof(uint64_t)); /* sentence starts */
  uint64_t* en = (uint64_t*)malloc(cap * sizeof(uint64_t)); /* sentence ends   */
  if (!st || !en) { free(v); free(st); free(en); return -1; }
  tw_t t = {out, n, 0, 0, 0};
  t.width = unif(&s, 72, 88);
  while (t.pos < n) {
    if (ns == cap) {
      cap *= 2;
      uint64_t* a = (uint64_t*)realloc(st, cap * sizeof(uint64_t));
      uint64_t* b = (uint64_t*)realloc(en, cap * sizeof(uint64_t));
      if (!a || !b) { free(v); free(a ? a : st); free(b ? b : en); return -1; }
      st = a; en = b;
    }
    if (t.pos > 0) tw_sep(&t, &s);
    uint64_t start = t.pos;
    if (ns > 0 && u01(&s) < 0.2) { /* re-emit an earlier sentence verbatim */
      double g = lognormal(&s, log(65536.0), 2.0);
      if (g < 1) g = 1;
      if (g > (double)t.pos) g = (double)t.pos;
      uint64_t target = t.pos - (uint64_t)g;
      uint64_t lo = 0, hi = ns; /* latest sentence start <= target */
      while (lo + 1 < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (st[mid] <= target) lo = mid; else hi = mid;
      }
      for (uint64_t q = st[lo]; q < en[lo] && t.pos < n; q++) tw_put(&t, out[q]);
    } else {
      uint64_t words = geom(&s, 14.0);
      for (uint64_t w = 0; w < words && t.pos < n; w++) {
        if (w > 0) tw_sep(&t, &s);
        int id = zipf_word(v, &s);
        for (unsigned i = 0; i < v->len[id]; i++) tw_put(&t, (uint8_t)v->w[id][i]);
        if (w + 1 < words && u01(&s) < 0.08) tw_put(&t, ',');
      }
      double u = u01(&s);
      tw_put(&t, u < 0.9 ? '.' : u < 0.95 ? '?' : '!');
    }
    st[ns] = start;
    en[ns] = t.pos;
    ns++;
  }
  free(v); free(st); free(en);
  return 0;
}

/* -------------------------------------------------------------- proteins --- */

static const uint8_t AMINO[20] = {'A', 'C', 'D', 'E', 'F', 'G', 'H', 'I', 'K', 'L',
                                  'M', 'N', 'P', 'Q', 'R', 'S', 'T', 'V', 'W', 'Y'};

/* Residue from a cumulative background distribution. */
static uint8_t amino_draw(const double* cum, uint64_t* s) {
  double u = u01(s);
  int k = 0;
  while (k < 19 && u >= cum[k]) k++;
  return AMINO[k];
}

/* Protein-like sequences, one per line: lengths Lognormal(ln 350, 0.6)
 * clipped to [30, 5000]; residues order-0 from a background drawn once per
 * seed (Dirichlet(2, ..., 2) over the 20 amino acids).  A new sequence is,
 * with probability 0.30, a homolog of a uniformly chosen earlier sequence
 * (each residue substituted with probability 0.15, deleted with 0.01, a
 * random residue inserted after it with 0.01), with probability 0.05 an
 * exact duplicate of one, else fresh.  With probability 0.03 a sequence
 * carries a low-complexity segment: a unit of 1..3 residues repeated to
 * 10..60 residues at a uniform place. */
int axs_protein(uint8_t* out, uint64_t n, uint64_t seed) {
  uint64_t s = seed * 0x2545F4914F6CDD1DULL + 0x632BE59BD9B4E019ULL;
  double cum[20], t = 0, g[20];
  for (int k = 0; k < 20; k++) { /* Gamma(2,1) = -ln(u1 u2) */
    g[k] = -log((1.0 - u01(&s)) * (1.0 - u01(&s)));
    t += g[k];
  }
  double acc = 0;
  for (int k = 0; k < 20; k++) { acc += g[k] / t; cum[k] = acc; }
  cum[19] = 1.0;
  uint64_t cap = 1024, ns = 0;
  uint64_t* st = (uint64_t*)malloc(cap * sizeof(uint64_t));
  uint64_t* en = (uint64_t*)malloc(cap * sizeof(uint64_t));
  if (!st || !en) { free(st); free(en); return -1; }
  uint64_t pos = 0;
  while (pos < n) {
    if (ns == cap) {
      cap *= 2;
      uint64_t* a = (uint64_t*)realloc(st, cap * sizeof(uint64_t));
      uint64_t* b = (uint64_t*)realloc(en, cap * sizeof(uint64_t));
      if (!a || !b) { free(a ? a : st); free(b ? b : en); return -1; }
      st = a; en = b;
    }
    const uint64_t start = pos;
    const double u = u01(&s);
    if (ns > 0 && u < 0.35) {
      const uint64_t j = unif(&s, 0, ns - 1);
      const int exact = u >= 0.30;
      for (uint64_t q = st[j]; q < en[j] && pos < n; q++) {
        if (exact) { out[pos++] = out[q]; continue; }
        const double e = u01(&s);
        if (e < 0.01) continue; /* deletion */
        out[pos++] = e < 0.16 ? amino_draw(cum, &s) : out[q];
        if (pos < n && u01(&s) < 0.01) out[pos++] = amino_draw(cum, &s); /* insertion */
      }
    } else {
      double l = floor(lognormal(&s, log(350.0), 0.6) + 0.5);
      uint64_t len = l < 30 ? 30 : l > 5000 ? 5000 : (uint64_t)l;
      for (uint64_t k = 0; k < len && pos < n; k++) out[pos++] = amino_draw(cum, &s);
    }
    if (pos > start + 60 && u01(&s) < 0.03) { /* low-complexity segment */
      const unsigned period = (unsigned)unif(&s, 1, 3);
      uint8_t unit[3];
      for (unsigned k = 0; k < period; k++) unit[k] = amino_draw(cum, &s);
      const uint64_t len = unif(&s, 10, 60), at = unif(&s, start, pos - len);
      for (uint64_t k = 0; k < len; k++) out[at + k] = unit[k % period];
    }
    st[ns] = start;
    en[ns] = pos;
    ns++;
    if (pos < n) out[pos++] = '\n';
  }
  free(st); free(en);
  return 0;
}

/* ----------------------------------------------------------------- reads --- */

/* FASTQ-like sequencing reads of a synthetic genome.  The genome is the DNA
 * generator's output for this seed (N bases replaced by A, lowercase folded
 * to uppercase), of max(2^20, n / 32) bases, so the reads cover it about
 * twelve times.  Record i is "@r<i>/1", a 100-base read from a uniform
 * genome position (each base substituted with probability 0.005), "+" and
 * a quality line of Phred+33 symbols: a walk over levels 2..41 starting at
 * 38 that per base holds (0.5), steps up (0.25) or down (0.2) by one, or
 * jumps to a uniform level (0.05), and past base 70 drifts one level down
 * with probability 0.3. */
int axs_reads(uint8_t* out, uint64_t n, uint64_t seed) {
  uint64_t s = seed * 0x2545F4914F6CDD1DULL + 0x8CB92BA72F3D8DD7ULL;
  const uint64_t glen = n / 32 > (1u << 20) ? n / 32 : (1u << 20);
  uint8_t* g = (uint8_t*)malloc(glen);
  if (!g) return -1;
  if (axs_dna(g, glen, seed ^ 0x5EEDull)) { free(g); return -1; }
  for (uint64_t k = 0; k < glen; k++) g[k] = g[k] == 'N' || g[k] == 'n' ? 'A' : (uint8_t)(g[k] & ~0x20);
  const unsigned R = 100;
  uint64_t pos = 0, rec = 0;
  char head[32];
  while (pos < n) {
    int hl = 0;
    uint64_t v = rec++, d = 1;
    while (v / d >= 10) d *= 10;
    head[hl++] = '@';
    head[hl++] = 'r';
    for (; d; d /= 10) head[hl++] = (char)('0' + (v / d) % 10);
    head[hl++] = '/';
    head[hl++] = '1';
    head[hl++] = '\n';
    for (int k = 0; k < hl && pos < n; k++) out[pos++] = (uint8_t)head[k];
    const uint64_t at = unif(&s, 0, glen - R);
    for (unsigned k = 0; k < R && pos < n; k++) {
      uint8_t b = g[at + k];
      if (u01(&s) < 0.005) b = BASES[(base_code(b) + 1 + unif(&s, 0, 2)) & 3];
      out[pos++] = b;
    }
    if (pos < n) out[pos++] = '\n';
    if (pos < n) out[pos++] = '+';
    if (pos < n) out[pos++] = '\n';
    unsigned q = 38;
    for (unsigned k = 0; k < R && pos < n; k++) {
      const double u = u01(&s);
      if (u >= 0.95) q = (unsigned)unif(&s, 2, 41);
      else if (u >= 0.75) q = q > 2 ? q - 1 : 2;
      else if (u >= 0.5) q = q < 41 ? q + 1 : 41;
      if (k > 70 && q > 2 && u01(&s) < 0.3) q--;
      out[pos++] = (uint8_t)(33 + q);
    }
    if (pos < n) out[pos++] = '\n';
  }
  free(g);
  return 0;
}

/* ---------------------------------------------------------- batch plan --- */

void axs_batch_plan(uint32_t count, uint64_t seed, uint64_t* sizes, uint8_t* kinds) {
  uint64_t s = seed * 0x2545F4914F6CDD1DULL + 0x632BE59BD9B4E019ULL;
  for (uint32_t i = 0; i < count; i++) {
    kinds[i] = u01(&s) < 0.6 ? 0 : 1;
    double z = lognormal(&s, log(1048576.0), 1.2);
    if (z < 65536.0) z = 65536.0;
    if (z > 67108864.0) z = 67108864.0;
    sizes[i] = (uint64_t)z;
  }
}

/* --------------------------------------------------------------- trace --- */

static uint64_t zipf_small(uint64_t* s, const double* cum, uint64_t k) {
  double u = u01(s);
  uint64_t lo = 0, hi = k - 1;
  while (lo < hi) {
    uint64_t mid = (lo + hi) / 2;
    if (cum[mid] < u) lo = mid + 1; else hi = mid;
  }
  return lo;
}

void axs_trace(uint64_t count, uint64_t seed, uint64_t n, uint32_t block, double rate,
               uint64_t len_min, uint64_t len_max,
               uint64_t* arrival_ns, uint64_t* off, uint64_t* len) {
  uint64_t s = seed * 0x2545F4914F6CDD1DULL + 0x3C6EF372FE94F82BULL;
  enum { CENTRES = 1024, DMAX = 4096 };
  double cc[CENTRES], cd[DMAX + 1];
  double acc = 0;
  for (int i = 0; i < CENTRES; i++) { acc += pow(i + 1.0, -1.1); cc[i] = acc; }
  for (int i = 0; i < CENTRES; i++) cc[i] /= acc;
  acc = 0;
  for (int i = 0; i <= DMAX; i++) { acc += pow(i + 1.0, -1.1); cd[i] = acc; }
  for (int i = 0; i <= DMAX; i++) cd[i] /= acc;
  uint64_t centre[CENTRES];
  for (int i = 0; i < CENTRES; i++) centre[i] = n ? unif(&s, 0, n - 1) : 0;
  double t = 0;
  for (uint64_t r = 0; r < count; r++) {
    t += -log(1.0 - u01(&s)) / rate;
    arrival_ns[r] = (uint64_t)(t * 1e9);
    uint64_t L = len_min;
    if (len_max > len_min) L = (uint64_t)exp(log((double)len_min) + u01(&s) * (log((double)len_max) - log((double)len_min)));
    if (L > n) L = n;
    len[r] = L;
    uint64_t span = n - L; /* start in [0, span] */
    uint64_t o;
    if (u01(&s) < 0.8) {
      uint64_t c = centre[zipf_small(&s, cc, CENTRES)];
      int64_t d = (int64_t)zipf_small(&s, cd, DMAX + 1);
      if (u01(&s) < 0.5) d = -d;
      int64_t base = (int64_t)(c / block) + d;
      int64_t p = base * (int64_t)block + (int64_t)unif(&s, 0, block - 1);
      if (p < 0) p = 0;
      if ((uint64_t)p > span) p = (int64_t)span;
      o = (uint64_t)p;
    } else {
      o = unif(&s, 0, span);
    }
    off[r] = o;
  }
}
