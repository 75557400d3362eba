/*
 * Plain CPU oracle for canonical k-mer counting (KMC 2, Deorowicz et al.).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (the plain definition the paper's method reaches exactly):
 *   the set of pairs (K, c) where K ranges over the canonical k-mers of every
 *   window of every read that holds only A/C/G/T, and c is the number of such
 *   windows; a pair is kept iff cutoff_min <= c <= cutoff_max; pairs are
 *   listed in ascending K.
 *
 * Paper passages followed:
 *   - symbol code A->0 C->1 G->2 T->3, leftmost symbol most significant
 *     (supplement, database [map] example and .kmc_suf packing example);
 *   - canonical k-mer = the smaller of the k-mer and its reverse complement
 *     (Methods, "Minimizers of k-mers");
 *   - cutoffs: k-mers counted fewer than ci or more than cx times are not
 *     written (supplement, -ci / -cx options and the min_count / max_count
 *     header fields);
 *   - signature of a k-mer = the smallest canonical m-mer that neither starts
 *     with AAA nor with ACA and has no AA anywhere except at its beginning
 *     (Methods, "From minimizers to signatures"); a k-mer with no such m-mer
 *     takes the extra value 4^m (the database map has 4^m + 1 entries).
 *
 * Readings where the paper is silent: bytes other than A/C/G/T (either case)
 * are invalid and exclude every window that holds one; palindromic k-mers
 * count once per occurrence; counts are exact 32-bit values.
 *
 * Keys are held as unsigned __int128 so that one code path serves every k in
 * [1, 64]; the result is returned in the library's table layout: key_words = 1
 * (k <= 32) or 2 (hi word first, then lo word).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* A/C/G/T in either case -> 0..3, anything else -> -1. */
static int sym_code(uint8_t b) {
  switch (b) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

/* Forward value F = sum_t code[t] * 4^(k-1-t) and reverse-complement value
 * R = sum_t (3 - code[t]) * 4^t of the k symbols at s; returns min(F, R), or
 * F alone when canonical is 0 (the supplement's -b option: k-mers counted as
 * read, not in canonical form).  The caller guarantees the k symbols are
 * valid. */
static u128 key_at(const uint8_t* s, uint32_t k, int canonical) {
  u128 f = 0, r = 0, pw = 1;
  for (uint32_t t = 0; t < k; ++t) {
    int c = sym_code(s[t]);
    f = f * 4 + (u128)c;
    r = r + (u128)(3 - c) * pw;
    pw *= 4;
  }
  if (!canonical) return f;
  return f < r ? f : r;
}

/* ---------------------------------------------------------------- count -- */

static int cmp_u128(const void* a, const void* b) {
  u128 x = *(const u128*)a, y = *(const u128*)b;
  return (x > y) - (x < y);
}

typedef struct {
  u128* keys;      /* this partition's keys */
  uint64_t n;
  uint32_t ci, cx;
  /* results: run-length counted, cutoff-filtered */
  u128* out_keys;
  uint32_t* out_counts;
  uint64_t n_out;
} part_t;

static void* sort_and_count(void* arg) {
  part_t* P = (part_t*)arg;
  qsort(P->keys, P->n, sizeof(u128), cmp_u128);
  P->out_keys = (u128*)malloc((P->n ? P->n : 1) * sizeof(u128));
  P->out_counts = (uint32_t*)malloc((P->n ? P->n : 1) * sizeof(uint32_t));
  P->n_out = 0;
  if (!P->out_keys || !P->out_counts) {  /* the caller sees the NULL and fails */
    free(P->out_keys);
    free(P->out_counts);
    P->out_keys = NULL;
    P->out_counts = NULL;
    return NULL;
  }
  uint64_t m = 0;
  uint64_t i = 0;
  while (i < P->n) {
    uint64_t j = i + 1;
    while (j < P->n && P->keys[j] == P->keys[i]) ++j;
    uint64_t c = j - i;
    if (c >= P->ci && c <= P->cx) {
      P->out_keys[m] = P->keys[i];
      P->out_counts[m] = (uint32_t)c;
      ++m;
    }
    i = j;
  }
  P->n_out = m;
  return NULL;
}

typedef struct { part_t* parts; int first, step, count; } job_t;

static void* worker(void* arg) {
  job_t* J = (job_t*)arg;
  for (int q = J->first; q < J->count; q += J->step) sort_and_count(&J->parts[q]);
  return NULL;
}

/* Run fn(args + i * size) for i in [0, n) on n threads (inline where a
 * thread cannot be created). */
static void run_threads(void* (*fn)(void*), void* args, size_t size, int n) {
  pthread_t th[256];
  int created[256] = {0};
  if (n > 256) n = 256;
  for (int t = 0; t < n; ++t) {
    void* a = (char*)args + (size_t)t * size;
    if (n > 1 && pthread_create(&th[t], NULL, fn, a) == 0)
      created[t] = 1;
    else
      fn(a);
  }
  for (int t = 0; t < n; ++t)
    if (created[t]) pthread_join(th[t], NULL);
}

/* Number of valid windows of reads [r0, r1): for every maximal run of valid
 * bytes of length L inside one read, max(0, L - k + 1). */
static uint64_t valid_windows_range(const uint8_t* seq, const uint64_t* offsets,
                                    uint64_t r0, uint64_t r1, uint32_t k) {
  uint64_t total = 0;
  for (uint64_t r = r0; r < r1; ++r) {
    uint64_t run = 0;
    for (uint64_t x = offsets[r]; x < offsets[r + 1]; ++x) {
      if (sym_code(seq[x]) >= 0) {
        ++run;
      } else {
        if (run >= k) total += run - k + 1;
        run = 0;
      }
    }
    if (run >= k) total += run - k + 1;
  }
  return total;
}

/* Number of valid windows of the whole input.  This is the closed form the
 * full count must sum to when cutoff_min <= 1 and cutoff_max is unbounded. */
uint64_t kmc_oracle_valid_windows(const uint8_t* seq, const uint64_t* offsets,
                                  uint64_t n_reads, uint32_t k) {
  return valid_windows_range(seq, offsets, 0, n_reads, k);
}

/* One thread's share of the enumeration: reads [r0, r1). */
typedef struct {
  const uint8_t* seq;
  const uint64_t* offsets;
  uint64_t r0, r1;
  uint32_t k, shift;
  uint32_t slice_bits;  /* 0: every key; else only keys whose top slice_bits */
  uint64_t slice;       /* bits of the 2k-bit key equal slice */
  int canonical;
  int n_parts;
  uint64_t n_win;   /* valid windows of the share */
  u128* keys;       /* the share's keys go to keys[0 .. n_win) */
  uint64_t* hist;   /* keys of the share per partition (n_parts) */
  uint64_t* pos;    /* next slot of each partition in `sorted` */
  u128* sorted;
} enum_t;

/* Is key K (2k bits) in the share's slice? */
static int in_slice(const enum_t* E, u128 K) {
  return E->slice_bits == 0 || (uint64_t)(K >> (2 * E->k - E->slice_bits)) == E->slice;
}

/* Every window of the share whose k bytes are all valid, in read order:
 * with keys == NULL only counted (of the slice), else its canonical key to
 * keys[] when it is in the slice, with the partition histogram.  Returns the
 * number of keys. */
static uint64_t enum_windows(enum_t* E, u128* keys) {
  const uint32_t k = E->k;
  uint64_t n = 0;
  for (uint64_t r = E->r0; r < E->r1; ++r) {
    uint64_t b = E->offsets[r], e = E->offsets[r + 1];
    if (e - b < k) continue;
    for (uint64_t j = b; j + k <= e; ++j) {
      int ok = 1;
      for (uint32_t t = 0; t < k; ++t)
        if (sym_code(E->seq[j + t]) < 0) { ok = 0; break; }
      if (!ok) continue;
      const u128 K = key_at(E->seq + j, k, E->canonical);
      if (!in_slice(E, K)) continue;
      if (keys) {
        keys[n] = K;
        if (E->n_parts > 1) E->hist[(uint32_t)(K >> E->shift)]++;
      }
      ++n;
    }
  }
  return n;
}

static void* enum_count(void* arg) {
  enum_t* E = (enum_t*)arg;
  E->n_win = E->slice_bits ? enum_windows(E, NULL)
                           : valid_windows_range(E->seq, E->offsets, E->r0, E->r1, E->k);
  return NULL;
}

/* Steps 1-2 on the share: every window whose k bytes are all valid ->
 * canonical key; and the partition histogram of the keys. */
static void* enum_keys(void* arg) {
  enum_t* E = (enum_t*)arg;
  enum_windows(E, E->keys);
  return NULL;
}

/* The share's keys to their partitions. */
static void* enum_scatter(void* arg) {
  enum_t* E = (enum_t*)arg;
  for (uint64_t i = 0; i < E->n_win; ++i) {
    const u128 K = E->keys[i];
    E->sorted[E->pos[(uint32_t)(K >> E->shift)]++] = K;
  }
  return NULL;
}

/* Enumerate every canonical k-mer, sort, run-length count, apply cutoffs.
 * With slice_bits > 0 only the keys whose top slice_bits bits (of the 2k-bit
 * key) equal slice are kept from the enumeration on: the result is the part
 * of the whole count in that key range, for inputs whose whole count would
 * not fit in memory (a key's count does not depend on the other keys).
 * n_threads > 1 splits the reads into n_threads consecutive shares that are
 * enumerated in parallel, partitions the keys by their top 8 bits (so
 * partitions are key ranges in order) and sorts each partition on its own
 * thread.  Returns 0 on success, -1 on bad arguments, -2 on allocation
 * failure (nothing allocated is left behind).  *out_keys and *out_counts are
 * malloc'd; release them with kmc_oracle_free. */
int kmc_oracle_count_slice(const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads,
                           uint32_t k, uint32_t cutoff_min, uint32_t cutoff_max, int canonical,
                           int n_threads, uint32_t slice_bits, uint64_t slice, uint64_t* out_n,
                           uint64_t** out_keys, uint32_t** out_counts) {
  if (k < 1 || k > 64 || !out_n || !out_keys || !out_counts) return -1;
  if (slice_bits > 2 * k || slice_bits > 32 || (slice_bits && slice >> slice_bits)) return -1;
  if (cutoff_min > cutoff_max) return -1;
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  const uint32_t ci = cutoff_min == 0 ? 1 : cutoff_min;
  const int n_parts = n_threads > 1 ? 256 : 1;
  const uint32_t shift = 2 * k > 8 ? 2 * k - 8 : 0;
  int rc = -2;
  uint64_t n = 0;

  enum_t* E = (enum_t*)calloc(n_threads, sizeof(enum_t));
  uint64_t* hist = (uint64_t*)calloc((size_t)n_threads * n_parts * 2, sizeof(uint64_t));
  uint64_t* cnt = (uint64_t*)calloc(n_parts + 1, sizeof(uint64_t));
  part_t* parts = (part_t*)calloc(n_parts, sizeof(part_t));
  job_t* jobs = (job_t*)calloc(n_threads, sizeof(job_t));
  u128* keys = NULL;
  u128* sorted = NULL;
  uint64_t* ok_keys = NULL;
  uint32_t* ok_counts = NULL;
  if (!E || !hist || !cnt || !parts || !jobs) goto done;

  /* Steps 1-2: the windows of each share, then every share's keys in place
   * (shares in read order, so single- and multi-threaded runs enumerate the
   * same sequence of keys). */
  for (int t = 0; t < n_threads; ++t) {
    E[t].seq = seq;
    E[t].offsets = offsets;
    E[t].r0 = n_reads * (uint64_t)t / (uint64_t)n_threads;
    E[t].r1 = n_reads * (uint64_t)(t + 1) / (uint64_t)n_threads;
    E[t].k = k;
    E[t].canonical = canonical;
    E[t].shift = shift;
    E[t].slice_bits = slice_bits;
    E[t].slice = slice;
    E[t].n_parts = n_parts;
    E[t].hist = hist + (size_t)t * n_parts;
    E[t].pos = hist + (size_t)(n_threads + t) * n_parts;
  }
  run_threads(enum_count, E, sizeof(enum_t), n_threads);
  for (int t = 0; t < n_threads; ++t) n += E[t].n_win;
  keys = (u128*)malloc((n ? n : 1) * sizeof(u128));
  if (!keys) goto done;
  {
    uint64_t before = 0;
    for (int t = 0; t < n_threads; ++t) {
      E[t].keys = keys + before;
      before += E[t].n_win;
    }
  }
  run_threads(enum_keys, E, sizeof(enum_t), n_threads);

  /* Step 3: partition by the top 8 bits of the 2k-bit key (one partition
   * when single-threaded), then sort and count each partition. */
  if (n_parts > 1) {
    sorted = (u128*)malloc((n ? n : 1) * sizeof(u128));
    if (!sorted) goto done;
    for (int q = 0; q < n_parts; ++q)
      for (int t = 0; t < n_threads; ++t) cnt[q + 1] += E[t].hist[q];
    for (int q = 0; q < n_parts; ++q) cnt[q + 1] += cnt[q];
    /* share t's keys of partition q follow those of shares 0 .. t-1 */
    for (int q = 0; q < n_parts; ++q) {
      uint64_t at = cnt[q];
      for (int t = 0; t < n_threads; ++t) {
        E[t].pos[q] = at;
        at += E[t].hist[q];
      }
    }
    for (int t = 0; t < n_threads; ++t) E[t].sorted = sorted;
    run_threads(enum_scatter, E, sizeof(enum_t), n_threads);
    free(keys);
    keys = NULL;
  } else {
    sorted = keys;
    keys = NULL;
    cnt[1] = n;
  }
  for (int q = 0; q < n_parts; ++q) {
    parts[q].keys = sorted + cnt[q];
    parts[q].n = cnt[q + 1] - cnt[q];
    parts[q].ci = ci;
    parts[q].cx = cutoff_max;
  }
  /* static round-robin of partitions over threads */
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].parts = parts;
    jobs[t].first = t;
    jobs[t].step = n_threads;
    jobs[t].count = n_parts;
  }
  run_threads(worker, jobs, sizeof(job_t), n_parts > 1 ? n_threads : 1);
  for (int q = 0; q < n_parts; ++q)
    if (!parts[q].out_keys || !parts[q].out_counts) goto done;

  /* Step 4: concatenate the partitions in key order. */
  {
    uint64_t total = 0;
    for (int q = 0; q < n_parts; ++q) total += parts[q].n_out;
    const uint32_t kw = k <= 32 ? 1 : 2;
    ok_keys = (uint64_t*)malloc((total ? total : 1) * kw * sizeof(uint64_t));
    ok_counts = (uint32_t*)malloc((total ? total : 1) * sizeof(uint32_t));
    if (!ok_keys || !ok_counts) goto done;
    uint64_t m = 0;
    for (int q = 0; q < n_parts; ++q) {
      for (uint64_t i = 0; i < parts[q].n_out; ++i, ++m) {
        const u128 K = parts[q].out_keys[i];
        if (kw == 1) {
          ok_keys[m] = (uint64_t)K;
        } else {
          ok_keys[2 * m] = (uint64_t)(K >> 64);
          ok_keys[2 * m + 1] = (uint64_t)K;
        }
        ok_counts[m] = parts[q].out_counts[i];
      }
    }
    *out_n = total;
    *out_keys = ok_keys;
    *out_counts = ok_counts;
    ok_keys = NULL;
    ok_counts = NULL;
    rc = 0;
  }
done:
  if (parts)
    for (int q = 0; q < n_parts; ++q) {
      free(parts[q].out_keys);
      free(parts[q].out_counts);
    }
  free(ok_keys);
  free(ok_counts);
  free(keys);
  free(sorted);
  free(parts);
  free(jobs);
  free(cnt);
  free(hist);
  free(E);
  return rc;
}

/* The whole count: every key. */
int kmc_oracle_count(const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads,
                     uint32_t k, uint32_t cutoff_min, uint32_t cutoff_max, int canonical,
                     int n_threads, uint64_t* out_n, uint64_t** out_keys,
                     uint32_t** out_counts) {
  return kmc_oracle_count_slice(seq, offsets, n_reads, k, cutoff_min, cutoff_max, canonical,
                                n_threads, 0, 0, out_n, out_keys, out_counts);
}

void kmc_oracle_free(void* p) { free(p); }

/* ------------------------------------------------------------ signature -- */

/* Is the canonical m-mer whose symbols are s[0..m-1] (leftmost first) allowed
 * as a signature?  Not allowed: it starts with AAA, it starts with ACA, or it
 * has AA at any offset other than 0 (Methods, "From minimizers to
 * signatures").  filter == 0 allows every m-mer (plain canonical minimizers,
 * Methods, "Minimizers of k-mers"). */
static int mmer_allowed(const int* s, uint32_t m, int filter) {
  if (!filter) return 1;
  if (m >= 3 && s[0] == 0 && s[1] == 0 && s[2] == 0) return 0;
  if (m >= 3 && s[0] == 0 && s[1] == 1 && s[2] == 0) return 0;
  for (uint32_t i = 1; i + 1 < m; ++i)
    if (s[i] == 0 && s[i + 1] == 0) return 0;
  return 1;
}

/* Signature of the k-mer whose symbols are sym[0..k-1]: the minimum, over
 * the k-m+1 positions, of the canonical m-mer there, among allowed ones;
 * 4^m when no m-mer is allowed.  Plain O(k*m) per k-mer. */
static uint32_t signature_of_symbols(const int* sym, uint32_t k, uint32_t m, int filter) {
  uint32_t best = 1u << (2 * m); /* 4^m */
  int can[32];
  for (uint32_t i = 0; i + m <= k; ++i) {
    uint32_t f = 0, r = 0, pw = 1;
    for (uint32_t t = 0; t < m; ++t) {
      f = f * 4 + (uint32_t)sym[i + t];
      r = r + (uint32_t)(3 - sym[i + t]) * pw;
      pw *= 4;
    }
    uint32_t c = f < r ? f : r;
    for (uint32_t t = 0; t < m; ++t) can[t] = (int)((c >> (2 * (m - 1 - t))) & 3);
    if (mmer_allowed(can, m, filter) && c < best) best = c;
  }
  return best;
}

/* Signature of each packed key (library table layout, key_words words per
 * key).  Used to check on which bin the GPU path placed each k-mer.
 * m must be in [1, 15] and m <= k.  Returns 0, or -1 on bad arguments. */
int kmc_oracle_key_signatures(const uint64_t* keys, uint64_t n, uint32_t key_words,
                              uint32_t k, uint32_t m, int filter, uint32_t* out) {
  if (k < 1 || k > 64 || m < 1 || m > 15 || m > k) return -1;
  if (key_words != (k <= 32 ? 1u : 2u)) return -1;
  int sym[64];
  for (uint64_t i = 0; i < n; ++i) {
    u128 K = key_words == 1 ? (u128)keys[i]
                            : (((u128)keys[2 * i]) << 64) | (u128)keys[2 * i + 1];
    for (uint32_t t = 0; t < k; ++t) sym[t] = (int)((K >> (2 * (k - 1 - t))) & 3);
    out[i] = signature_of_symbols(sym, k, m, filter);
  }
  return 0;
}

/* Signature of the window starting at every byte position of the input:
 * out[j] = signature of the k bytes at j if they lie in one read and are all
 * valid, else 0xFFFFFFFF.  out has offsets[n_reads] entries.  The signature
 * is computed from the window's own symbols (either orientation gives the
 * same value, since the canonical m-mers of a k-mer and of its reverse
 * complement coincide). */
int kmc_oracle_window_signatures(const uint8_t* seq, const uint64_t* offsets,
                                 uint64_t n_reads, uint32_t k, uint32_t m, int filter,
                                 uint32_t* out) {
  if (k < 1 || k > 64 || m < 1 || m > 15 || m > k) return -1;
  int sym[64];
  for (uint64_t r = 0; r < n_reads; ++r) {
    uint64_t b = offsets[r], e = offsets[r + 1];
    for (uint64_t j = b; j < e; ++j) {
      out[j] = 0xFFFFFFFFu;
      if (j + k > e) continue;
      int ok = 1;
      for (uint32_t t = 0; t < k; ++t) {
        sym[t] = sym_code(seq[j + t]);
        if (sym[t] < 0) { ok = 0; break; }
      }
      if (ok) out[j] = signature_of_symbols(sym, k, m, filter);
    }
  }
  return 0;
}

/* ----------------------------------------------------------- count keys -- */

/* Occurrences of given canonical keys: every valid window of every read is
 * turned into its canonical key (forward and reverse-complement values rolled
 * one symbol at a time: F = F*4 + c mod 4^k, R = R/4 + (3-c)*4^(k-1)) and
 * looked up in an open-addressing table of the query keys.  Used to check
 * sampled entries of tables too large for a full sort.  keys: n_keys keys of
 * key_words words (hi word first for 2).  Returns 0, or -1 / -2 as above. */
typedef struct {
  const uint8_t* seq;
  const uint64_t* offsets;
  uint64_t r0, r1;
  uint32_t k;
  const u128* table;
  const uint32_t* slot_of;
  uint64_t mask;
  uint64_t* counts;
} ck_job_t;

static uint64_t mix_u128(u128 x) {
  uint64_t h = (uint64_t)x * 0x9E3779B97F4A7C15ull ^ (uint64_t)(x >> 64) * 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ull;
  return h ^ (h >> 32);
}

static void* count_keys_worker(void* arg) {
  ck_job_t* J = (ck_job_t*)arg;
  const uint32_t k = J->k;
  const u128 kmask = k == 64 ? ~(u128)0 : (((u128)1 << (2 * k)) - 1);
  const u128 EMPTY = ~(u128)0;
  for (uint64_t r = J->r0; r < J->r1; ++r) {
    u128 f = 0, rc = 0;
    uint64_t run = 0;
    for (uint64_t x = J->offsets[r]; x < J->offsets[r + 1]; ++x) {
      const int c = sym_code(J->seq[x]);
      if (c < 0) {
        run = 0;
        continue;
      }
      f = ((f << 2) | (u128)c) & kmask;
      rc = (rc >> 2) | ((u128)(3 - c) << (2 * k - 2));
      if (++run < k) continue;
      const u128 key = f < rc ? f : rc;
      uint64_t s = mix_u128(key) & J->mask;
      while (J->table[s] != EMPTY) {
        if (J->table[s] == key) {
          J->counts[J->slot_of[s]]++;
          break;
        }
        s = (s + 1) & J->mask;
      }
    }
  }
  return NULL;
}

int kmc_oracle_count_keys(const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads,
                          uint32_t k, const uint64_t* keys, uint64_t n_keys,
                          uint32_t key_words, int n_threads, uint64_t* counts_out) {
  if (k < 1 || k > 64 || (key_words != 1 && key_words != 2) || !counts_out) return -1;
  if (n_keys && !keys) return -1;
  uint64_t cap = 16;
  while (cap < 2 * n_keys + 16) cap <<= 1;
  u128* table = (u128*)malloc(cap * sizeof(u128));
  uint32_t* slot_of = (uint32_t*)malloc(cap * sizeof(uint32_t));
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 64) n_threads = 64;
  uint64_t* part = (uint64_t*)calloc((size_t)n_threads * (n_keys + 1), sizeof(uint64_t));
  if (!table || !slot_of || !part) {
    free(table);
    free(slot_of);
    free(part);
    return -2;
  }
  for (uint64_t s = 0; s < cap; ++s) table[s] = ~(u128)0;
  for (uint64_t i = 0; i < n_keys; ++i) {
    const u128 key = key_words == 1 ? (u128)keys[i]
                                    : (((u128)keys[2 * i] << 64) | (u128)keys[2 * i + 1]);
    uint64_t s = mix_u128(key) & (cap - 1);
    while (table[s] != ~(u128)0 && table[s] != key) s = (s + 1) & (cap - 1);
    table[s] = key;  /* a repeated query key shares the slot of its first copy */
    slot_of[s] = (uint32_t)i;
  }
  pthread_t th[64];
  ck_job_t jobs[64];
  int created[64] = {0};
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].seq = seq;
    jobs[t].offsets = offsets;
    jobs[t].r0 = n_reads * (uint64_t)t / (uint64_t)n_threads;
    jobs[t].r1 = n_reads * (uint64_t)(t + 1) / (uint64_t)n_threads;
    jobs[t].k = k;
    jobs[t].table = table;
    jobs[t].slot_of = slot_of;
    jobs[t].mask = cap - 1;
    jobs[t].counts = part + (size_t)t * (n_keys + 1);
    if (n_threads > 1 && pthread_create(&th[t], NULL, count_keys_worker, &jobs[t]) == 0)
      created[t] = 1;
    else
      count_keys_worker(&jobs[t]);
  }
  for (int t = 0; t < n_threads; ++t)
    if (created[t]) pthread_join(th[t], NULL);
  for (uint64_t i = 0; i < n_keys; ++i) {
    uint64_t c = 0;
    for (int t = 0; t < n_threads; ++t) c += part[(size_t)t * (n_keys + 1) + i];
    counts_out[i] = c;
  }
  /* repeated query keys: every copy reports the count */
  for (uint64_t i = 0; i < n_keys; ++i) {
    const u128 key = key_words == 1 ? (u128)keys[i]
                                    : (((u128)keys[2 * i] << 64) | (u128)keys[2 * i + 1]);
    uint64_t s = mix_u128(key) & (cap - 1);
    while (table[s] != key) s = (s + 1) & (cap - 1);
    counts_out[i] = counts_out[slot_of[s]];
  }
  free(table);
  free(slot_of);
  free(part);
  return 0;
}
