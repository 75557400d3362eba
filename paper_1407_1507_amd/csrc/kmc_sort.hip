// Sorting phase, second half: sort every tile of keys in LDS, count runs of
// equal keys, apply the cutoffs and compact the kept (key, count) pairs; then
// assemble the per-tile outputs into one table.
//
// Method (KMC 2, Methods, "Sketch of the algorithm" and "Additional
// features"): the extracted k-mers of a bin are radix sorted; equal keys are
// then adjacent and their run length is the k-mer's count; a k-mer is written
// only if cutoff_min <= count <= cutoff_max, decided here where the total
// count is known.
//
// Tile counting (a persistent workgroup per compute-unit slot, one tile at
// a time, the tile's keys in registers): every key goes into an LDS hash
// table whose per-slot counter ends equal to the run length a sort would
// give it; the slots are read back, the cutoffs applied, and only the kept
// keys are put in key order (a rank sort, or a counting pass on the key digit
// below their common prefix).  64-bit keys claim slots by a 64-bit
// compare-and-swap; 128-bit keys by a fingerprint, with the full key beside
// it and a check that no two keys of the tile share one.  Tiles above the
// tile limit, and 128-bit tiles whose fingerprints clash, take most-
// significant-digit passes through HBM (8-bit digits) until their pieces
// fit, and the pieces are counted the same way (128-bit pieces by hashed
// buckets sorted in LDS).
#include <algorithm>
#include <atomic>

#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

namespace {

template <int KW> struct SortCfg;
// CAP: keys a workgroup holds; DIRECT: largest tile the tile kernel counts
// itself (64-bit keys: the LDS hash table at load <= 3/4), larger ones go to
// the big-tile kernel, whose register budget is its own.
template <> struct SortCfg<1> {
  static constexpr uint32_t CAP = kTileCap1, DIG = 12, ITEMS = kTileCap1 / kSortThreads;
  static constexpr uint32_t DIRECT = 3 * kTileCap1 / 4;
};
template <> struct SortCfg<2> {
  static constexpr uint32_t CAP = kTileCap2, DIG = 11, ITEMS = kTileCap2 / kSortThreads;
  static constexpr uint32_t DIRECT = 3 * kTileCap2 / 4;
};
constexpr uint32_t kInsMax = 16;    // mixed buckets up to this size: insertion sort by one lane
constexpr uint32_t kBigMax = 256;   // larger mixed buckets listed per tile (CAP / (kInsMax + 1) < 256)

__device__ __forceinline__ uint64_t load_key(const uint64_t* p, uint64_t i, uint64_t*) { return p[i]; }
__device__ __forceinline__ u128 load_key(const uint64_t* p, uint64_t i, u128*) {
  return ((u128)p[2 * i] << 64) | p[2 * i + 1];
}
__device__ __forceinline__ void store_key(uint64_t* p, uint64_t i, uint64_t v) { p[i] = v; }
__device__ __forceinline__ void store_key(uint64_t* p, uint64_t i, u128 v) {
  p[2 * i] = (uint64_t)(v >> 64);
  p[2 * i + 1] = (uint64_t)v;
}

__device__ __forceinline__ uint64_t wave_and(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v &= __shfl_xor(v, d, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
  return v;
}

// Block-wide AND and OR of per-thread values (identity for threads with no
// key: all ones / zero).  red needs 4 * (blockDim.x / 64) u64 words.
template <class K>
__device__ void block_and_or(K& a, K& o, uint64_t* red) {
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint64_t a0 = wave_and((uint64_t)a), o0 = wave_or((uint64_t)o);
  uint64_t a1 = 0, o1 = 0;
  if (sizeof(K) == 16) {
    a1 = wave_and((uint64_t)((u128)a >> 64));
    o1 = wave_or((uint64_t)((u128)o >> 64));
  }
  if (lane == 0) {
    red[wid] = a0;
    red[nw + wid] = o0;
    red[2 * nw + wid] = a1;
    red[3 * nw + wid] = o1;
  }
  __syncthreads();
  a0 = ~0ull; o0 = 0; a1 = ~0ull; o1 = 0;
  for (uint32_t w = 0; w < nw; ++w) {
    a0 &= red[w];
    o0 |= red[nw + w];
    a1 &= red[2 * nw + w];
    o1 |= red[3 * nw + w];
  }
  __syncthreads();
  if (sizeof(K) == 16) {
    a = (K)(((u128)a1 << 64) | a0);
    o = (K)(((u128)o1 << 64) | o0);
  } else {
    a = (K)a0;
    o = (K)o0;
  }
}

// Cross-lane exchange of a key within a wave.
__device__ __forceinline__ uint64_t shfl_xor_key(uint64_t v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ u128 shfl_xor_key(u128 v, int m) {
  const uint64_t lo = __shfl_xor((uint64_t)v, m, 64), hi = __shfl_xor((uint64_t)(v >> 64), m, 64);
  return ((u128)hi << 64) | lo;
}

// Sort A[s, e) (e - s <= 64 R) with one wave: bitonic network over 64 R
// slots (slot i = 64 r + lane, padding sorts last as the all-ones key).
// Distances >= 64 compare two registers of a lane, smaller ones two lanes.
template <class K, int R>
__device__ void wave_bitonic(K* A, uint32_t s, uint32_t e) {
  const uint32_t lane = threadIdx.x & 63u;
  K v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = s + r * 64 + lane;
    v[r] = i < e ? A[i] : ~K(0);
  }
  constexpr uint32_t N = 64u * R;
#pragma unroll
  for (uint32_t size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (uint32_t j = size >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        const int rj = (int)(j / 64);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int q = r ^ rj;
          if (q > r) {
            const bool asc = (((uint32_t)r * 64 + lane) & size) == 0;
            const K a = v[r], b = v[q];
            const bool sw = asc ? (a > b) : (a < b);
            v[r] = sw ? b : a;
            v[q] = sw ? a : b;
          }
        }
      } else {
        const bool lower = (lane & j) == 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const K o = shfl_xor_key(v[r], (int)j);
          const bool asc = (((uint32_t)r * 64 + lane) & size) == 0;
          const K mn = v[r] < o ? v[r] : o, mx = v[r] < o ? o : v[r];
          v[r] = (asc == lower) ? mn : mx;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = s + r * 64 + lane;
    if (i < e) A[i] = v[r];
  }
}

__device__ __forceinline__ uint32_t high_bit(uint64_t x) { return 63u - __clzll(x); }
__device__ __forceinline__ uint32_t high_bit(u128 x) {
  const uint64_t hi = (uint64_t)(x >> 64);
  return hi ? 127u - __clzll(hi) : 63u - __clzll((uint64_t)x);
}

constexpr uint32_t kRankMax = 256;  // kept keys ordered by a rank sort, at most

// Output slot of every kept (distinct) 128-bit key of K[0, kept), kept <=
// kRankMax: the number of smaller kept keys (for 64-bit keys one lane per key
// measured faster).  K holds the all-ones key (never
// canonical) from kept up to the next multiple of 8.  Up to four lanes share
// a key, each counting over a part of K, so that a small set is spread over
// the whole workgroup; emit(i, key, slot) runs once per key.  All threads
// call it.
template <class K, class Emit>
__device__ __forceinline__ void rank_kept(const K* keys, uint32_t kept, Emit emit) {
  const uint32_t tid = threadIdx.x;
  const uint32_t p = kept <= kSortThreads / 4 ? 4u : kept <= kSortThreads / 2 ? 2u : 1u;
  const uint32_t span = ((kept + 7) & ~7u) / p;  // even
  const uint32_t i = tid / p, part = tid % p;
  uint32_t r = 0;
  K x = 0;
  if (i < kept) {
    x = keys[i];
    for (uint32_t j = part * span, e = j + span; j < e; j += 2)
      r += (uint32_t)(keys[j] < x) + (uint32_t)(keys[j + 1] < x);
  }
  if (p >= 2) r += __shfl_xor(r, 1, 64);  // the lanes of a key are adjacent in a wave
  if (p >= 4) r += __shfl_xor(r, 2, 64);
  if (i < kept && part == 0) emit(i, x, r);
}

// LDS carve-up of the tile sort.  128-bit keys keep the hashed-bucket
// counting path (mixed buckets, big-bucket list); 64-bit keys only take the
// hash table and keep a small separate area for the kept keys instead.
template <int KW>
struct SortShared {
  typedef typename KeyOf<KW>::T K;
  K A[SortCfg<KW>::CAP];
  uint32_t H[((1u << SortCfg<KW>::DIG) > SortCfg<KW>::CAP ? (1u << SortCfg<KW>::DIG)
                                                           : SortCfg<KW>::CAP) + 1];
  uint32_t mixed[(1u << SortCfg<KW>::DIG) / 32];  // bit d: bucket d holds > 1 distinct key
  uint64_t red[4 * kSortThreads / 64];
  uint32_t tmp[kSortThreads / 64];
  uint16_t big[kBigMax];
  uint32_t nbig;
};
template <>
struct SortShared<1> {
  uint64_t A[SortCfg<1>::CAP];      // hash table keys (~0: empty)
  uint32_t H[SortCfg<1>::CAP + 1];  // hash table counters
  uint64_t K2[kRankMax];            // kept keys of a tile, in read-back order
  uint32_t C2[kRankMax];
  uint64_t red[4 * kSortThreads / 64];
  uint32_t tmp[kSortThreads / 64];
};

__device__ __forceinline__ uint32_t hash_top(uint64_t x, uint32_t t) {
  return (uint32_t)((x * 0x9E3779B97F4A7C15ull) >> (64 - t));
}
__device__ __forceinline__ uint32_t hash_top(u128 x, uint32_t t) {
  return hash_top((uint64_t)((uint64_t)x ^ ((uint64_t)(x >> 64) * 0xD6E8FEB86659FD93ull)), t);
}
__device__ __forceinline__ uint32_t bit_len(uint32_t x) { return 32u - __clz(x); }

// Order the kept (distinct) keys held in registers (key[m], cnt[m] > 0) and
// write them ascending to out_keys / out_counts: compact them into A / H, one
// counting pass on the key digit below their common prefix (diff = AND ^ OR
// of the kept keys), then each key's slot is its bucket start plus the number
// of smaller keys in its bucket.  kbase = this thread's first compacted slot.
// All threads call it; A / H must no longer be read by anyone.
template <int KW>
__device__ void order_kept(typename KeyOf<KW>::T (&key)[SortCfg<KW>::ITEMS],
                           uint32_t (&cnt)[SortCfg<KW>::ITEMS], uint32_t kbase, uint32_t kept,
                           typename KeyOf<KW>::T diff, uint64_t* out_keys,
                           uint32_t* out_counts, typename KeyOf<KW>::T* A, uint32_t* H,
                           uint32_t* tmp) {
  typedef typename KeyOf<KW>::T K;
  constexpr uint32_t ITEMS = SortCfg<KW>::ITEMS, DIG = SortCfg<KW>::DIG;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  // ---- order the kept keys (distinct) by a key-digit counting pass.
  // Kept runs are first compacted into A / H (both free now), so the loops
  // below run over ceil(kept / threads) slots instead of all register slots.
  {
    uint32_t at = kbase;
#pragma unroll
    for (uint32_t qq = 0; qq < ITEMS; ++qq) {
      if (cnt[qq]) {
        A[at] = key[qq];
        H[at] = cnt[qq];
        ++at;
      }
    }
  }
  __syncthreads();
  const uint32_t mk = (kept + nt - 1) / nt;  // uniform
  const uint32_t hb = high_bit(diff);
  const uint32_t t2 = min(min(DIG, bit_len(kept) + 1), hb + 1);
  const uint32_t shift = hb + 1 - t2;
  const uint32_t nb2 = 1u << t2, dmask = nb2 - 1;
#pragma unroll
  for (uint32_t m = 0; m < ITEMS; ++m) {
    cnt[m] = 0;
    if (m < mk) {
      const uint32_t i = m * nt + tid;
      if (i < kept) {
        key[m] = A[i];
        cnt[m] = H[i];
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < nb2; i += nt) H[i] = 0;
  __syncthreads();
#pragma unroll
  for (uint32_t m = 0; m < ITEMS; ++m)
    if (m < mk && cnt[m]) atomicAdd(&H[(uint32_t)(key[m] >> shift) & dmask], 1u);
  __syncthreads();
  block_exclusive_scan(H, nb2, tmp);
#pragma unroll
  for (uint32_t m = 0; m < ITEMS; ++m)
    if (m < mk && cnt[m]) A[atomicAdd(&H[(uint32_t)(key[m] >> shift) & dmask], 1u)] = key[m];
  __syncthreads();
#pragma unroll
  for (uint32_t m = 0; m < ITEMS; ++m) {
    if (m < mk && cnt[m]) {
      const uint32_t d = (uint32_t)(key[m] >> shift) & dmask;
      const uint32_t s = d ? H[d - 1] : 0, e = H[d];
      uint32_t r = s;
      for (uint32_t j = s; j < e; ++j) r += A[j] < key[m];
      store_key(out_keys, r, key[m]);
      out_counts[r] = cnt[m];
    }
  }
  __syncthreads();
}

template <int KW>
__device__ __forceinline__ uint32_t count_tile(typename KeyOf<KW>::T (&key)[SortCfg<KW>::ITEMS], uint32_t n,
                               uint64_t* out_keys, uint32_t* out_counts, uint32_t ci,
                               uint32_t cx, SortShared<KW>& S, uint32_t* distinct);

// Count a tile of 64-bit keys (n <= 3/4 of the table) with an LDS hash table:
// open addressing with linear probing over the A (keys) / H (counters) arrays;
// a key's first insertion claims an empty slot by compare-and-swap and every
// occurrence adds one to that slot's counter, so each counter ends equal to
// the run length a sort of the tile would give that key.  The all-ones key
// marks an empty slot: it is never canonical (its reverse complement, all A,
// is smaller).
//
// kClean: the table is empty on entry, and is left empty on return (slots
// are cleared as they are read back, and whatever the ordering step below
// writes is cleared after it), so a persistent workgroup initialises it once.
// Kept keys (at most kRankMax of them) are put in key order by a rank sort:
// each one counts the kept keys smaller than itself; more kept keys take the
// digit-counting order of order_kept.
template <bool kClean>
__device__ __forceinline__ uint32_t hash_finish(uint64_t (&key)[SortCfg<1>::ITEMS],
                                                uint64_t* out_keys, uint32_t* out_counts,
                                                uint32_t ci, uint32_t cx, SortShared<1>& S,
                                                uint32_t* distinct);

//
// kW: key m carries the weight wt[m] (a run of wt[m] equal keys); a slot's
// counter then sums the weights of its key.
template <bool kClean, bool kW = false>
__device__ __forceinline__ uint32_t count_tile_hash(uint64_t (&key)[SortCfg<1>::ITEMS], uint32_t n,
                                                    uint64_t* out_keys, uint32_t* out_counts,
                                                    uint32_t ci, uint32_t cx, SortShared<1>& S,
                                                    uint32_t* distinct,
                                                    const uint32_t* wt = nullptr) {
  constexpr uint32_t ITEMS = SortCfg<1>::ITEMS, T = SortCfg<1>::CAP, TB = 12;
  static_assert((1u << TB) == T, "table size");
  constexpr uint64_t EMPTY = ~0ull;
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t nt = kSortThreads;  // every launch of the tile kernels
  if (!kClean) {
    for (uint32_t s = tid; s < T; s += nt) {
      S.A[s] = EMPTY;
      S.H[s] = 0;
    }
    __syncthreads();
  }
  // A wave has few partners to hide LDS latency behind (the table limits a
  // compute unit to three workgroups), so the first probes of G keys are
  // issued before any result is awaited, and the read-back issues all its
  // loads at once: one LDS round trip per group instead of one per key.
  constexpr uint32_t G = 4;
#pragma unroll
  for (uint32_t g = 0; g < ITEMS; g += G) {
    if (g * nt < n) {  // uniform
      uint64_t old[G];
      uint32_t slot[G];
#pragma unroll
      for (uint32_t u = 0; u < G; ++u) {
        slot[u] = hash_top(key[g + u], TB);
        old[u] = 0;
        if ((g + u) * nt + tid < n)
          old[u] = atomicCAS(reinterpret_cast<unsigned long long*>(&S.A[slot[u]]),
                             (unsigned long long)EMPTY, (unsigned long long)key[g + u]);
      }
#pragma unroll
      for (uint32_t u = 0; u < G; ++u) {
        if ((g + u) * nt + tid < n) {
          uint32_t sl = slot[u];
          uint64_t ov = old[u];
          while (ov != EMPTY && ov != key[g + u]) {  // linear probing on a clash
            sl = (sl + 1) & (T - 1);
            ov = atomicCAS(reinterpret_cast<unsigned long long*>(&S.A[sl]),
                           (unsigned long long)EMPTY, (unsigned long long)key[g + u]);
          }
          atomicAdd(&S.H[sl], kW ? wt[g + u] : 1u);
        }
      }
    }
  }
  __syncthreads();
  return hash_finish<kClean>(key, out_keys, out_counts, ci, cx, S, distinct);
}

// The second half of count_tile_hash, once every key is in the table: read
// back (and clear) every slot, apply the cutoffs and write the kept keys in
// key order.  key is scratch.  All threads call it.
template <bool kClean>
__device__ __forceinline__ uint32_t hash_finish(uint64_t (&key)[SortCfg<1>::ITEMS],
                                                uint64_t* out_keys, uint32_t* out_counts,
                                                uint32_t ci, uint32_t cx, SortShared<1>& S,
                                                uint32_t* distinct) {
  constexpr uint32_t ITEMS = SortCfg<1>::ITEMS, T = SortCfg<1>::CAP;
  constexpr uint64_t EMPTY = ~0ull;
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t nt = kSortThreads;
  // read back (and clear) every slot; an empty slot reads count 0 < ci
  uint32_t cnt[ITEMS];
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {  // T == ITEMS * threads
    const uint32_t s = i * nt + tid;
    key[i] = S.A[s];
    cnt[i] = S.H[s];
  }
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {
    const uint32_t s = i * nt + tid;
    S.A[s] = EMPTY;
    S.H[s] = 0;
  }
  uint32_t nh = 0, nk = 0;
  uint64_t a = ~0ull, o = 0;
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {
    const uint32_t c = cnt[i];
    nh += c != 0;
    const bool keep = c >= ci && c <= cx;
    cnt[i] = keep ? c : 0u;
    if (keep) {
      a &= key[i];
      o |= key[i];
      ++nk;
    }
  }
  // distinct keys (high half) and kept keys (low half) in one scan; both
  // are at most CAP, so the halves never carry into each other
  uint32_t both;
  const uint32_t pre = block_scan_one((nh << 16) | nk, S.tmp, both);  // read-back is done
  *distinct = both >> 16;
  const uint32_t kept = both & 0xFFFFu, kbase = pre & 0xFFFFu;
  if (kept == 0) return 0;
  if (kept <= kRankMax) {
    // kept keys to their own small area (the table is already empty again),
    // then every kept key's output slot is the number of smaller kept keys
    uint32_t at = kbase;
#pragma unroll
    for (uint32_t i = 0; i < ITEMS; ++i) {
      if (cnt[i]) {
        S.K2[at] = key[i];
        S.C2[at] = cnt[i];
        ++at;
      }
    }
    __syncthreads();
    if (tid < kept) {
      const uint64_t x = S.K2[tid];
      uint32_t r = 0;
      for (uint32_t j = 0; j < kept; ++j) r += S.K2[j] < x;
      out_keys[r] = x;
      out_counts[r] = S.C2[tid];
    }
    // K2 is written again only after the next tile's barriers
    return kept;
  }
  block_and_or<uint64_t>(a, o, S.red);
  const uint64_t diff = a ^ o;  // nonzero: more than one key is kept
  order_kept<1>(key, cnt, kbase, kept, diff, out_keys, out_counts, S.A, S.H, S.tmp);
  if (kClean) {
    // order_kept used A[0, kept) and H[0, max(kept, buckets)), buckets <= T
    const uint32_t hb = high_bit(diff);
    const uint32_t t2 = min(min(SortCfg<1>::DIG, bit_len(kept) + 1), hb + 1);
    const uint32_t used = max(kept, 1u << t2);
    for (uint32_t s = tid; s < kept; s += nt) S.A[s] = EMPTY;
    for (uint32_t s = tid; s < used; s += nt) S.H[s] = 0;
    __syncthreads();
  }
  return kept;
}

// ------------------------------------------------- 128-bit keys: hash table
// LDS compare-and-swap is 64 bits wide, so a 128-bit key claims its slot by
// a 48-bit fingerprint (with a 16-bit count in the same word) and the claimer
// stores the full key beside it.  After the inserts every key checks the key
// stored in its slot: if two different keys shared a fingerprint the tile is
// not counted here (the caller hands it to the exact big-tile path), so the
// result never depends on the fingerprint.
constexpr uint32_t kHashSlots2 = 2048, kHashBits2 = 11;
static_assert((1u << kHashBits2) == kHashSlots2 && kHashSlots2 == kTileCap2, "table size");

struct HashShared2 {
  uint64_t F[kHashSlots2];  // 0: empty; else fingerprint << 16 | count
  u128 K[kHashSlots2];      // the key of an occupied slot
  uint32_t C2[kRankMax];    // counts of the kept keys (keys in K[0, kept))
  uint64_t red[4 * kSortThreads / 64];
  uint32_t tmp[kSortThreads / 64];
  // the occupied slots, in claiming order (a tile holds at most DIRECT keys)
  uint16_t L[3 * kHashSlots2 / 4];
  uint32_t n_claimed;
};
// three workgroups per compute unit
static_assert(3 * sizeof(HashShared2) <= 160 * 1024, "LDS of the 128-bit tile kernel");

__device__ __forceinline__ uint64_t mix128(u128 x) {
  uint64_t h = (uint64_t)x * 0x9E3779B97F4A7C15ull ^ (uint64_t)(x >> 64) * 0xD6E8FEB86659FD93ull;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  return h;
}

constexpr uint32_t kFingerprintClash = 0xFFFFFFFFu;

// Returns the kept count, or kFingerprintClash (nothing written, table
// empty again).  The table is empty on entry and on return.
// fp_mask keeps the fingerprint's low bits (47 in use; fewer only to let tests
// force clashes).
__device__ uint32_t count_tile_hash2(u128 (&key)[SortCfg<2>::ITEMS], uint32_t n,
                                     uint64_t* out_keys, uint32_t* out_counts, uint32_t ci,
                                     uint32_t cx, uint64_t fp_mask, HashShared2& S,
                                     uint32_t* distinct) {
  constexpr uint32_t ITEMS = SortCfg<2>::ITEMS, T = kHashSlots2;
  static_assert(T == ITEMS * kSortThreads, "one slot per register slot");
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t nt = kSortThreads;  // every launch of the tile kernels
  // As for 64-bit keys: the first probes of G keys go out before any result
  // is awaited, and the checks and the read-back issue all their loads at once.
  constexpr uint32_t G = 4;
  uint32_t slot_of[ITEMS];
#pragma unroll
  for (uint32_t g = 0; g < ITEMS; g += G) {
    if (g * nt < n) {  // uniform
      uint64_t old[G], fp[G];
#pragma unroll
      for (uint32_t u = 0; u < G; ++u) {
        const uint64_t h = mix128(key[g + u]);
        slot_of[g + u] = (uint32_t)(h >> (64 - kHashBits2));
        fp[u] = (h & fp_mask) | (1ull << 47);  // never 0
        old[u] = 0;
        if ((g + u) * nt + tid < n)
          old[u] = atomicCAS(reinterpret_cast<unsigned long long*>(&S.F[slot_of[g + u]]), 0ull,
                             (unsigned long long)((fp[u] << 16) | 1u));
      }
#pragma unroll
      for (uint32_t u = 0; u < G; ++u) {
        if ((g + u) * nt + tid < n) {
          uint32_t slot = slot_of[g + u];
          uint64_t ov = old[u];
          while (ov != 0 && (ov >> 16) != fp[u]) {  // linear probing on a clash
            slot = (slot + 1) & (T - 1);
            ov = atomicCAS(reinterpret_cast<unsigned long long*>(&S.F[slot]), 0ull,
                           (unsigned long long)((fp[u] << 16) | 1u));
          }
          if (ov == 0) {
            S.K[slot] = key[g + u];
            S.L[atomicAdd(&S.n_claimed, 1u)] = (uint16_t)slot;
          } else {
            atomicAdd(reinterpret_cast<unsigned long long*>(&S.F[slot]), 1ull);
          }
          slot_of[g + u] = slot;
        }
      }
    }
  }
  __syncthreads();
  const uint32_t nd = S.n_claimed;  // distinct keys (slots claimed)
  bool clash = false;
#pragma unroll
  for (uint32_t m = 0; m < ITEMS; ++m)
    if (m * nt + tid < n && S.K[slot_of[m]] != key[m]) clash = true;
  const bool any_clash = __syncthreads_or(clash);  // every thread has read nd
  if (tid == 0) S.n_claimed = 0;  // the barriers below order this before the next tile
  if (any_clash) {
    for (uint32_t i = tid; i < T; i += nt) S.F[i] = 0;
    __syncthreads();
    return kFingerprintClash;
  }
  // read back (and clear) the claimed slots only (at most DIRECT: the first
  // RB entries of each thread); the other entries count 0
  constexpr uint32_t RB = (SortCfg<2>::DIRECT + nt - 1) / nt;
  uint32_t cnt[ITEMS];
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {
    const uint32_t j = i * nt + tid;
    cnt[i] = 0;
    if (i < RB && i * nt < nd && j < nd) {
      const uint32_t s = S.L[j];
      const uint64_t w = S.F[s];
      key[i] = S.K[s];
      cnt[i] = (uint32_t)(w & 0xFFFFu);
      S.F[s] = 0;
    }
  }
  uint32_t nh = 0, nk = 0;
  u128 a = ~(u128)0, o = 0;
#pragma unroll
  for (uint32_t i = 0; i < ITEMS; ++i) {
    const uint32_t c = cnt[i];
    nh += c != 0;
    const bool keep = c >= ci && c <= cx;
    cnt[i] = keep ? c : 0u;
    if (keep) {
      a &= key[i];
      o |= key[i];
      ++nk;
    }
  }
  // distinct keys (high half) and kept keys (low half) in one scan
  uint32_t both;
  const uint32_t pre = block_scan_one((nh << 16) | nk, S.tmp, both);  // read-back is done
  *distinct = both >> 16;
  const uint32_t kept = both & 0xFFFFu, kbase = pre & 0xFFFFu;
  if (kept == 0) return 0;
  if (kept <= kRankMax) {
    // kept keys into K (free once read back), counts beside; each kept key's
    // output slot is the number of smaller kept keys
    uint32_t at = kbase;
#pragma unroll
    for (uint32_t i = 0; i < ITEMS; ++i) {
      if (cnt[i]) {
        S.K[at] = key[i];
        S.C2[at] = cnt[i];
        ++at;
      }
    }
    if (tid >= kept && tid < ((kept + 7) & ~7u)) S.K[tid] = ~(u128)0;  // never canonical
    __syncthreads();
    rank_kept(S.K, kept, [&](uint32_t i, const u128& x, uint32_t r) {
      store_key(out_keys, r, x);
      out_counts[r] = S.C2[i];
    });
    __syncthreads();  // the next tile's inserts write K
    return kept;
  }
  block_and_or<u128>(a, o, S.red);
  const u128 diff = a ^ o;  // nonzero: more than one key is kept
  // kept keys are ordered in K with counts in F's words, which are cleared
  // again afterwards
  uint32_t* H = reinterpret_cast<uint32_t*>(S.F);
  order_kept<2>(key, cnt, kbase, kept, diff, out_keys, out_counts, S.K, H, S.tmp);
  const uint32_t hb = high_bit(diff);
  const uint32_t t2 = min(min(SortCfg<2>::DIG, bit_len(kept) + 1), hb + 1);
  const uint32_t dirty = max(kept, 1u << t2);
  for (uint32_t i = tid; i < (dirty + 1) / 2; i += nt) S.F[i] = 0;
  __syncthreads();
  return kept;
}

// Count a tile whose keys are in registers: the hash table for 64-bit keys
// (up to CAP keys: the table has CAP slots, so every distinct key finds one),
// hashed buckets for 128-bit keys.
template <int KW>
__device__ __forceinline__ uint32_t count_any(typename KeyOf<KW>::T (&key)[SortCfg<KW>::ITEMS],
                                              uint32_t n, uint64_t* out_keys,
                                              uint32_t* out_counts, uint32_t ci, uint32_t cx,
                                              SortShared<KW>& S, uint32_t* distinct);
template <>
__device__ __forceinline__ uint32_t count_any<1>(uint64_t (&key)[SortCfg<1>::ITEMS], uint32_t n,
                                                 uint64_t* out_keys, uint32_t* out_counts,
                                                 uint32_t ci, uint32_t cx, SortShared<1>& S,
                                                 uint32_t* distinct) {
  return count_tile_hash<false>(key, n, out_keys, out_counts, ci, cx, S, distinct);
}

// The tile kernel's counting: only the hash table for 64-bit keys (tiles up
// to DIRECT keys), so the kernel carries none of the bucket path's registers;
// the kernel keeps the table empty between tiles.
template <bool kW = false>
__device__ __forceinline__ uint32_t count_direct(uint64_t (&key)[SortCfg<1>::ITEMS], uint32_t n,
                                                 uint64_t* out_keys, uint32_t* out_counts,
                                                 uint32_t ci, uint32_t cx, SortShared<1>& S,
                                                 uint32_t* distinct, const uint32_t* wt = nullptr) {
  return count_tile_hash<true, kW>(key, n, out_keys, out_counts, ci, cx, S, distinct, wt);
}
__device__ __forceinline__ uint32_t count_direct(u128 (&key)[SortCfg<2>::ITEMS], uint32_t n,
                                                 uint64_t* out_keys, uint32_t* out_counts,
                                                 uint32_t ci, uint32_t cx, SortShared<2>& S,
                                                 uint32_t* distinct) {
  return count_tile<2>(key, n, out_keys, out_counts, ci, cx, S, distinct);
}
template <>
__device__ __forceinline__ uint32_t count_any<2>(u128 (&key)[SortCfg<2>::ITEMS], uint32_t n,
                                                 uint64_t* out_keys, uint32_t* out_counts,
                                                 uint32_t ci, uint32_t cx, SortShared<2>& S,
                                                 uint32_t* distinct) {
  return count_tile<2>(key, n, out_keys, out_counts, ci, cx, S, distinct);
}

template <int KW>
__device__ __forceinline__ void load_tile(const uint64_t* src, uint32_t n,
                                          typename KeyOf<KW>::T (&key)[SortCfg<KW>::ITEMS]) {
#pragma unroll
  for (uint32_t m = 0; m < SortCfg<KW>::ITEMS; ++m) {
    const uint32_t i = m * blockDim.x + threadIdx.x;
    if (i < n) key[m] = load_key(src, i, (typename KeyOf<KW>::T*)nullptr);
  }
}

__device__ __forceinline__ void load_weights(const uint32_t* src, uint32_t n,
                                             uint32_t (&w)[SortCfg<1>::ITEMS]) {
#pragma unroll
  for (uint32_t m = 0; m < SortCfg<1>::ITEMS; ++m) {
    const uint32_t i = m * blockDim.x + threadIdx.x;
    if (i < n) w[m] = src[i];
  }
}

// kW (64-bit keys): key i carries the weight wsrc[i].
template <int KW, bool kW = false>
__device__ uint32_t sort_count_emit(const uint64_t* src, const uint32_t* wsrc, uint32_t n,
                                    uint64_t* out_keys, uint32_t* out_counts, uint32_t ci,
                                    uint32_t cx, SortShared<KW>& S, uint32_t* distinct) {
  typename KeyOf<KW>::T key[SortCfg<KW>::ITEMS];
  load_tile<KW>(src, n, key);
  if constexpr (KW == 1 && kW) {
    uint32_t w[SortCfg<1>::ITEMS];
    load_weights(wsrc, n, w);
    return count_tile_hash<false, true>(key, n, out_keys, out_counts, ci, cx, S, distinct, w);
  } else {
    return count_any<KW>(key, n, out_keys, out_counts, ci, cx, S, distinct);
  }
}

// Same as sort_count_emit, with the tile's keys already in registers
// (key[m] = key m * blockDim.x + threadIdx.x, for those < n); key is clobbered.
// Used for the pieces of 128-bit big tiles (64-bit keys always take the hash
// table).  Steps:
//   1. counting pass on a hashed digit (about one bucket per key): equal keys
//      share a bucket whatever the key distribution;
//   2. a bucket whose keys are not all equal to its first key is "mixed"; only
//      mixed buckets are sorted (insertion by a lane, bitonic by a wave,
//      rank sort by the workgroup above 256 keys);
//   3. runs of equal keys: in a bucket that is not mixed the run is the whole
//      bucket; counts, cutoffs; kept keys stay in registers;
//   4. the kept keys are put in key order by order_kept.
// Returns the kept count; *distinct receives the number of distinct keys.
template <int KW>
__device__ __forceinline__ uint32_t count_tile(typename KeyOf<KW>::T (&key)[SortCfg<KW>::ITEMS], uint32_t n,
                               uint64_t* out_keys, uint32_t* out_counts, uint32_t ci,
                               uint32_t cx, SortShared<KW>& S, uint32_t* distinct) {
  typedef typename KeyOf<KW>::T K;
  constexpr uint32_t ITEMS = SortCfg<KW>::ITEMS, DIG = SortCfg<KW>::DIG;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  uint32_t cnt[ITEMS];  // 0: not a kept run head

  // ---- 1. group equal keys by a hashed digit
  const uint32_t t = min(DIG, bit_len(n));
  const uint32_t nb = 1u << t;
  {
    uint32_t pos[ITEMS], hd[ITEMS];
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m)
      if (m * nt + tid < n) hd[m] = hash_top(key[m], t);
    for (uint32_t i = tid; i < nb; i += nt) S.H[i] = 0;
    for (uint32_t i = tid; i < (nb + 31) / 32; i += nt) S.mixed[i] = 0;
    if (tid == 0) S.nbig = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m)
      if (m * nt + tid < n) atomicAdd(&S.H[hd[m]], 1u);
    __syncthreads();
    block_exclusive_scan(S.H, nb, S.tmp);
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m) {
      if (m * nt + tid < n) {
        pos[m] = atomicAdd(&S.H[hd[m]], 1u);
        S.A[pos[m]] = key[m];
      }
    }
    __syncthreads();
    // ---- 2. S.H[d] is the end of bucket d; flag and sort the mixed buckets
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m) {
      if (m * nt + tid < n) {
        const uint32_t d = hd[m];
        if (S.A[d ? S.H[d - 1] : 0] != key[m]) atomicOr(&S.mixed[d >> 5], 1u << (d & 31));
      }
    }
    __syncthreads();
    // the lane holding a mixed bucket's first slot sorts it (or lists it)
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m) {
      if (m * nt + tid < n) {
        const uint32_t d = hd[m];
        const uint32_t s = d ? S.H[d - 1] : 0, e = S.H[d];
        if (pos[m] == s && ((S.mixed[d >> 5] >> (d & 31)) & 1u)) {
          if (e - s <= kInsMax) {
            for (uint32_t i = s + 1; i < e; ++i) {
              const K x = S.A[i];
              uint32_t j = i;
              while (j > s && S.A[j - 1] > x) {
                S.A[j] = S.A[j - 1];
                --j;
              }
              S.A[j] = x;
            }
          } else {
            S.big[atomicAdd(&S.nbig, 1u)] = (uint16_t)d;
          }
        }
      }
    }
    __syncthreads();
  }
  const uint32_t nbig = S.nbig;
  if (nbig) {
    const uint32_t wid = tid >> 6, nw = nt >> 6;
    for (uint32_t bb = wid; bb < nbig; bb += nw) {
      const uint32_t d = S.big[bb];
      const uint32_t s = d ? S.H[d - 1] : 0, e = S.H[d], sz = e - s;
      if (sz <= 64) wave_bitonic<K, 1>(S.A, s, e);
      else if (sz <= 128) wave_bitonic<K, 2>(S.A, s, e);
      else if (sz <= 256) wave_bitonic<K, 4>(S.A, s, e);
    }
    __syncthreads();
    for (uint32_t bb = 0; bb < nbig; ++bb) {
      const uint32_t d = S.big[bb];
      const uint32_t s = d ? S.H[d - 1] : 0, e = S.H[d];
      if (e - s <= 256) continue;
      K v[ITEMS];
      uint32_t rk[ITEMS];
#pragma unroll
      for (uint32_t m = 0; m < ITEMS; ++m) {
        const uint32_t i = s + m * nt + tid;
        if (i < e) {
          const K x = S.A[i];
          uint32_t r = 0;
          for (uint32_t j = s; j < e; ++j) {
            const K y = S.A[j];
            r += (y < x) || (y == x && j < i);
          }
          v[m] = x;
          rk[m] = r;
        }
      }
      __syncthreads();
#pragma unroll
      for (uint32_t m = 0; m < ITEMS; ++m)
        if (s + m * nt + tid < e) S.A[s + rk[m]] = v[m];
      __syncthreads();
    }
  }

  // ---- 3. run heads (equal keys never sit in two buckets, so a head is any
  // slot whose key differs from the previous slot's), counts, cutoffs;
  // kept runs stay in registers
  const uint32_t per2 = (n + nt - 1) / nt;
  const uint32_t b0 = min(n, tid * per2), b1 = min(n, b0 + per2);
  uint32_t nh = 0;
  for (uint32_t i = b0; i < b1; ++i) nh += (i == 0 || S.A[i] != S.A[i - 1]);
  uint32_t H_total;
  uint32_t h = block_scan_one(nh, S.tmp, H_total);
  for (uint32_t i = b0; i < b1; ++i)
    if (i == 0 || S.A[i] != S.A[i - 1]) S.H[h++] = i;
  if (tid == 0) S.H[H_total] = n;
  __syncthreads();
  *distinct = H_total;
  const uint32_t per3 = (H_total + nt - 1) / nt;  // <= ITEMS
  const uint32_t h0 = min(H_total, tid * per3), h1 = min(H_total, h0 + per3);
  K a = ~K(0), o = 0;
  uint32_t nk = 0;
#pragma unroll
  for (uint32_t qq = 0; qq < ITEMS; ++qq) {
    const uint32_t q = h0 + qq;
    cnt[qq] = 0;
    if (q < h1) {
      const uint32_t c = S.H[q + 1] - S.H[q];
      if (c >= ci && c <= cx) {
        key[qq] = S.A[S.H[q]];
        cnt[qq] = c;
        a &= key[qq];
        o |= key[qq];
        ++nk;
      }
    }
  }
  uint32_t kept;
  const uint32_t kbase = block_scan_one(nk, S.tmp, kept);  // barrier: A/H reads are done
  if (kept == 0) return 0;
  block_and_or<K>(a, o, S.red);
  const K diff = a ^ o;
  if (diff == 0) {  // a single kept key
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m)
      if (cnt[m]) {
        store_key(out_keys, 0, key[m]);
        out_counts[0] = cnt[m];
      }
    __syncthreads();
    return 1;
  }

  order_kept<KW>(key, cnt, kbase, kept, diff, out_keys, out_counts, S.A, S.H, S.tmp);
  __syncthreads();
  return kept;
}

// Persistent: the grid is the number of workgroups resident at once, and
// workgroup g takes tiles g, g + G, g + 2G, ... (tens of thousands of short
// tiles would otherwise be bound by workgroup dispatch).  kW: counts[i]
// holds the weight of key i on entry (the key stands for that many equal
// keys), and the counters sum weights.
template <int KW, bool kW>
__global__ void __launch_bounds__(kSortThreads, 3)  // 3 waves per SIMD: as many as LDS allows
k_tile_sort(KeyCfg kc, const Tile* __restrict__ tiles, uint64_t n_tiles, uint64_t* keys,
            uint32_t* counts, uint32_t* tile_out, uint32_t* big_list, uint64_t* big_off,
            uint32_t* n_big, unsigned long long* big_total, uint32_t* tile_distinct,
            uint32_t* big_size) {
  typedef typename KeyOf<KW>::T K;
  constexpr uint32_t ITEMS = SortCfg<KW>::ITEMS, CAP = SortCfg<KW>::CAP;
  static_assert(KW == 1 || !kW, "weights with 64-bit keys only");
  __shared__ SortShared<KW> S;
  if (KW == 1) {  // the hash table starts empty; count_direct leaves it empty
    for (uint32_t i = threadIdx.x; i < CAP; i += blockDim.x) {
      S.A[i] = ~K(0);
      S.H[i] = 0;
    }
    __syncthreads();
  }
  // the next tile's keys are loaded into registers while the current tile
  // is counted (double buffering hides the load latency behind the LDS work)
  auto direct = [](const Tile& x) { return x.size != 0 && x.size <= SortCfg<KW>::DIRECT; };
  Tile next = tiles[blockIdx.x];
  K nkey[ITEMS];
  uint32_t nw[kW ? ITEMS : 1];
  if (direct(next)) {
    load_tile<KW>(keys + next.begin * KW, next.size, nkey);
    if constexpr (kW) load_weights(counts + next.begin, next.size, nw);
  }
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const Tile T = next;
    K key[ITEMS];
    uint32_t w[kW ? ITEMS : 1];
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m) key[m] = nkey[m];
    if constexpr (kW) {
#pragma unroll
      for (uint32_t m = 0; m < ITEMS; ++m) w[m] = nw[m];
    }
    if (t + gridDim.x < n_tiles) {
      next = tiles[t + gridDim.x];
      if (direct(next)) {
        load_tile<KW>(keys + next.begin * KW, next.size, nkey);
        if constexpr (kW) load_weights(counts + next.begin, next.size, nw);
      }
    }
    if (T.size == 0) {
      if (threadIdx.x == 0) tile_out[t] = tile_distinct[t] = 0;
    } else if (T.size > SortCfg<KW>::DIRECT) {
      if (threadIdx.x == 0) {
        tile_out[t] = tile_distinct[t] = 0;
        const uint32_t idx = atomicAdd(n_big, 1u);
        big_list[idx] = (uint32_t)t;
        big_size[idx] = T.size;
        big_off[idx] = atomicAdd(big_total, (unsigned long long)T.size);  // own slice of tmp
      }
    } else {
      uint32_t d;
      uint32_t kept;
      if constexpr (kW)
        kept = count_direct<true>(key, T.size, keys + T.begin * KW, counts + T.begin,
                                  kc.cutoff_min, kc.cutoff_max, S, &d, w);
      else
        kept = count_direct(key, T.size, keys + T.begin * KW, counts + T.begin, kc.cutoff_min,
                            kc.cutoff_max, S, &d);
      if (threadIdx.x == 0) {
        tile_out[t] = kept;
        tile_distinct[t] = d;
      }
    }
  }
}

// Tiles of 128-bit keys: the fingerprint hash table; tiles above DIRECT keys
// and tiles whose fingerprints clash go to the big-tile kernel.  Persistent,
// like k_tile_sort.
__global__ void __launch_bounds__(kSortThreads, 3)
k_tile_hash2(KeyCfg kc, const Tile* __restrict__ tiles, uint64_t n_tiles, uint64_t* keys,
             uint32_t* counts, uint32_t* tile_out, uint32_t* big_list, uint64_t* big_off,
             uint32_t* n_big, unsigned long long* big_total, uint32_t* tile_distinct,
            uint32_t* big_size) {
  constexpr uint32_t ITEMS = SortCfg<2>::ITEMS;
  __shared__ HashShared2 S;
  for (uint32_t i = threadIdx.x; i < kHashSlots2; i += blockDim.x) S.F[i] = 0;
  if (threadIdx.x == 0) S.n_claimed = 0;
  __syncthreads();
  // the next tile's keys are loaded into registers while the current tile
  // is counted (double buffering)
  Tile next = tiles[blockIdx.x];
  u128 nkey[ITEMS];
  if (next.size != 0 && next.size <= SortCfg<2>::DIRECT)
    load_tile<2>(keys + next.begin * 2, next.size, nkey);
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const Tile T = next;
    uint32_t kept = kFingerprintClash, d = 0;
    const bool direct = T.size != 0 && T.size <= SortCfg<2>::DIRECT;
    u128 key[ITEMS];
#pragma unroll
    for (uint32_t m = 0; m < ITEMS; ++m) key[m] = nkey[m];
    if (t + gridDim.x < n_tiles) {
      next = tiles[t + gridDim.x];
      if (next.size != 0 && next.size <= SortCfg<2>::DIRECT)
        load_tile<2>(keys + next.begin * 2, next.size, nkey);
    }
    if (T.size == 0) {
      kept = 0;
    } else if (direct) {
      kept = count_tile_hash2(key, T.size, keys + T.begin * 2, counts + T.begin, kc.cutoff_min,
                              kc.cutoff_max, (1ull << kc.fp_bits) - 1, S, &d);
    }
    if (threadIdx.x == 0) {
      if (kept == kFingerprintClash) {
        tile_out[t] = tile_distinct[t] = 0;
        const uint32_t idx = atomicAdd(n_big, 1u);
        big_list[idx] = (uint32_t)t;
        big_size[idx] = T.size;
        big_off[idx] = atomicAdd(big_total, (unsigned long long)T.size);
      } else {
        tile_out[t] = kept;
        tile_distinct[t] = d;
      }
    }
  }
}

// ------------------------------------------------------ streamed big tiles
// A tile too large for registers often holds few distinct keys (at 30-40x
// coverage a key occurs tens of times): its keys are then streamed through
// the LDS hash table in chunks of kStreamChunk, each key read once, and the
// table is read back as for a small tile.  The distinct keys claimed so far
// are checked after every chunk: once more than DIRECT are claimed the attempt
// stops (false returned, the table left as it is: every user of the table
// sets it up first) and the caller partitions the tile instead.  A chunk
// holds T - DIRECT keys, so the table never fills and every probe ends.
// kW: key i carries the weight wsrc[i].
constexpr uint32_t kStreamItems = 4;
constexpr uint32_t kStreamChunk = kStreamItems * kSortThreads;
static_assert(SortCfg<1>::CAP - SortCfg<1>::DIRECT >= kStreamChunk, "a chunk never fills the table");

template <bool kW = false>
__device__ bool stream_count_hash(const uint64_t* src, const uint32_t* wsrc, uint64_t n,
                                  uint64_t* out_keys, uint32_t* out_counts, uint32_t ci,
                                  uint32_t cx, SortShared<1>& S, uint32_t* claims,
                                  uint32_t* distinct, uint32_t* kept) {
  constexpr uint32_t T = SortCfg<1>::CAP, TB = 12, U = kStreamItems;
  constexpr uint64_t EMPTY = ~0ull;
  const uint32_t tid = threadIdx.x;
  constexpr uint32_t nt = kSortThreads;
  for (uint32_t s = tid; s < T; s += nt) {
    S.A[s] = EMPTY;
    S.H[s] = 0;
  }
  if (tid == 0) *claims = 0;
  uint64_t cur[U];
  uint32_t cw[kW ? U : 1];
#pragma unroll
  for (uint32_t u = 0; u < U; ++u) {
    const uint64_t i = (uint64_t)u * nt + tid;
    cur[u] = i < n ? src[i] : EMPTY;
    if constexpr (kW) cw[u] = i < n ? wsrc[i] : 0u;
  }
  __syncthreads();
  bool ok = true;
  for (uint64_t base = 0; base < n; base += kStreamChunk) {
    // the next chunk's loads go out before this chunk's inserts
    uint64_t nxt[U];
    uint32_t nw[kW ? U : 1];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint64_t i = base + kStreamChunk + (uint64_t)u * nt + tid;
      nxt[u] = i < n ? src[i] : EMPTY;
      if constexpr (kW) nw[u] = i < n ? wsrc[i] : 0u;
    }
    uint64_t old[U];
    uint32_t slot[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      slot[u] = hash_top(cur[u], TB);
      old[u] = 0;
      if (cur[u] != EMPTY)
        old[u] = atomicCAS(reinterpret_cast<unsigned long long*>(&S.A[slot[u]]),
                           (unsigned long long)EMPTY, (unsigned long long)cur[u]);
    }
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      if (cur[u] != EMPTY) {
        uint32_t sl = slot[u];
        uint64_t ov = old[u];
        while (ov != EMPTY && ov != cur[u]) {  // linear probing on a clash
          sl = (sl + 1) & (T - 1);
          ov = atomicCAS(reinterpret_cast<unsigned long long*>(&S.A[sl]),
                         (unsigned long long)EMPTY, (unsigned long long)cur[u]);
        }
        mine += ov == EMPTY;  // this key claimed its slot
        if constexpr (kW)
          atomicAdd(&S.H[sl], cw[u]);
        else
          atomicAdd(&S.H[sl], 1u);
      }
    }
    // claims of the wave, one atomic per wave
    uint32_t w = mine;
    for (int d = 32; d >= 1; d >>= 1) w += __shfl_xor(w, d, 64);
    if ((tid & 63u) == 0 && w) atomicAdd(claims, w);
    __syncthreads();
    const uint32_t c = *claims;  // the same for every thread: read between two barriers
    __syncthreads();             // before the next chunk adds to it
    if (c > SortCfg<1>::DIRECT) {
      ok = false;
      break;
    }
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) cur[u] = nxt[u];
    if constexpr (kW) {
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) cw[u] = nw[u];
    }
  }
  if (!ok) return false;
  uint64_t key[SortCfg<1>::ITEMS];
  *kept = hash_finish<false>(key, out_keys, out_counts, ci, cx, S, distinct);
  return true;
}

// ------------------------------------------------------------- big tiles
// One workgroup per tile larger than LDS.  Depth-first over MSD pieces: a
// piece that fits LDS is sorted and emitted; a piece whose keys are all equal
// is one run; any other piece is partitioned on the 8 bits below its common
// prefix into the other buffer (same offsets) and its children are visited in
// key order, so the output stays in ascending order.  Output is written over
// the tile's own keys at a cursor that never passes the piece being read.
// f(x) for every key of src[0..n): each lane keeps U loads in flight (one
// workgroup walks the whole piece, so latency, not bandwidth, bounds a pass).
template <class K, int U, class F>
__device__ __forceinline__ void for_each_key(const uint64_t* src, uint32_t n, F f) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  for (uint32_t base = 0; base < n; base += nt * U) {
    K x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = base + u * nt + tid;
      if (i < n) x[u] = load_key(src, i, (K*)nullptr);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (base + u * nt + tid < n) f(x[u]);
  }
}

struct Level {
  uint64_t base;
  uint32_t next, nchild, buf, pad;
  uint32_t cs[257];
};
template <int KW> struct MaxLevels { static constexpr int N = KW == 1 ? 10 : 18; };

// One big tile, by the whole workgroup.  kStream (64-bit keys): the tile is
// first streamed through the LDS hash table, and partitioned only if it holds
// too many distinct keys.  kW (64-bit keys): counts[i] holds the weight of
// key i on entry; weights move with their keys through tmpw, and a run sums
// its weights.
template <int KW, bool kStream, bool kW>
__device__ void big_tile(const KeyCfg& kc, const Tile* __restrict__ tiles, uint32_t t,
                         uint64_t tmp_off, uint64_t* keys, uint64_t* tmp, uint32_t* counts,
                         uint32_t* tmpw, uint32_t* tile_out, uint32_t* tile_distinct,
                         unsigned long long* big_out) {
  typedef typename KeyOf<KW>::T K;
  __shared__ SortShared<KW> S;
  __shared__ Level L[MaxLevels<KW>::N];
  __shared__ uint32_t cur[256];
  __shared__ unsigned long long outc, dist;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const Tile T = tiles[t];
  if constexpr (KW == 1 && kStream) {
    __shared__ uint32_t claims;
    uint32_t d, kept;
    if (stream_count_hash<kW>(keys + T.begin, counts + T.begin, T.size, keys + T.begin,
                              counts + T.begin, kc.cutoff_min, kc.cutoff_max, S, &claims, &d,
                              &kept)) {
      if (tid == 0) {
        tile_out[t] = kept;
        tile_distinct[t] = d;
        atomicAdd(big_out, (unsigned long long)kept);
      }
      __syncthreads();
      return;
    }
  }
  uint64_t* bufs[2] = {keys + T.begin * KW, tmp + tmp_off * KW};
  uint32_t* wbufs[2] = {counts + T.begin, kW ? tmpw + tmp_off : nullptr};
  __shared__ unsigned long long wsum;
  if (tid == 0) {
    L[0].base = 0;
    L[0].next = 0;
    L[0].nchild = 1;
    L[0].buf = 0;
    L[0].cs[0] = 0;
    L[0].cs[1] = T.size;
    outc = 0;
    dist = 0;
  }
  __syncthreads();
  int depth = 0;
  while (depth >= 0) {
    const uint32_t c = L[depth].next, nch = L[depth].nchild;
    __syncthreads();
    if (c == nch) {
      --depth;
      continue;
    }
    // consecutive children that fit LDS together are sorted as one piece
    // (they are adjacent key ranges, adjacent in the buffer)
    uint32_t c2 = c + 1;
    if (L[depth].cs[c2] - L[depth].cs[c] <= SortCfg<KW>::CAP)
      while (c2 < nch && L[depth].cs[c2 + 1] - L[depth].cs[c] <= SortCfg<KW>::CAP) ++c2;
    if (tid == 0) L[depth].next = c2;
    const uint64_t off = L[depth].base + L[depth].cs[c];
    const uint32_t n = L[depth].cs[c2] - L[depth].cs[c];
    const uint32_t buf = L[depth].buf;
    const uint64_t* src = bufs[buf] + off * KW;
    __syncthreads();
    if (n == 0) continue;
    const unsigned long long oc = outc;
    if (n <= SortCfg<KW>::CAP) {
      uint32_t d;
      const uint32_t kept = sort_count_emit<KW, kW>(src, wbufs[buf] + off, n,
                                                    keys + (T.begin + oc) * KW,
                                                    counts + T.begin + oc, kc.cutoff_min,
                                                    kc.cutoff_max, S, &d);
      if (tid == 0) {
        outc = oc + kept;
        dist += d;
      }
      __syncthreads();
      continue;
    }
    constexpr int U = 16 / KW;
    K a = ~K(0), o = 0;
    for_each_key<K, U>(src, n, [&](const K& x) {
      a &= x;
      o |= x;
    });
    block_and_or<K>(a, o, S.red);
    const K diff = a ^ o;
    if (diff == 0) {
      // one key: its count is n, or the sum of its weights
      uint64_t run = n;
      if constexpr (kW) {
        if (tid == 0) wsum = 0;
        __syncthreads();
        const uint32_t* ws = wbufs[buf] + off;
        uint64_t v = 0;
        for (uint32_t i = tid; i < n; i += nt) v += ws[i];
        for (int dd = 32; dd >= 1; dd >>= 1) v += __shfl_xor(v, dd, 64);
        if ((tid & 63u) == 0) atomicAdd(&wsum, (unsigned long long)v);
        __syncthreads();
        run = wsum;
        __syncthreads();  // every thread has read wsum
      }
      const uint32_t rc = run > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)run;
      if (tid == 0) {
        if (rc >= kc.cutoff_min && rc <= kc.cutoff_max) {
          store_key(keys, T.begin + oc, a);
          counts[T.begin + oc] = rc;
          outc = oc + 1;
        }
        dist += 1;
      }
      __syncthreads();
      continue;
    }
    const uint32_t hb = high_bit(diff);
    const uint32_t bits = hb + 1 < 8 ? hb + 1 : 8;
    const uint32_t shift = hb + 1 - bits;
    const uint32_t nb = 1u << bits, dmask = nb - 1;
    for (uint32_t i = tid; i < 256; i += nt) cur[i] = 0;
    __syncthreads();
    for_each_key<K, U>(src, n, [&](const K& x) {
      atomicAdd(&cur[(uint32_t)(x >> shift) & dmask], 1u);
    });
    __syncthreads();
    const uint32_t total = block_exclusive_scan(cur, nb, S.tmp);
    const int nd = depth + 1;
    for (uint32_t i = tid; i < nb; i += nt) L[nd].cs[i] = cur[i];
    if (tid == 0) {
      L[nd].cs[nb] = total;
      L[nd].base = off;
      L[nd].next = 0;
      L[nd].nchild = nb;
      L[nd].buf = 1 - buf;
    }
    __syncthreads();
    uint64_t* dst = bufs[1 - buf] + off * KW;
    if constexpr (kW) {
      // weights move with their keys
      const uint32_t* ws = wbufs[buf] + off;
      uint32_t* wd = wbufs[1 - buf] + off;
      for (uint32_t base = 0; base < n; base += nt * U) {
        K x[U];
        uint32_t w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t i = base + u * nt + tid;
          if (i < n) {
            x[u] = load_key(src, i, (K*)nullptr);
            w[u] = ws[i];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (base + u * nt + tid < n) {
            const uint32_t at = atomicAdd(&cur[(uint32_t)(x[u] >> shift) & dmask], 1u);
            store_key(dst, at, x[u]);
            wd[at] = w[u];
          }
        }
      }
    } else {
      for_each_key<K, U>(src, n, [&](const K& x) {
        store_key(dst, atomicAdd(&cur[(uint32_t)(x >> shift) & dmask], 1u), x);
      });
    }
    __threadfence();
    __syncthreads();
    depth = nd;
  }
  if (tid == 0) {
    tile_out[t] = (uint32_t)outc;
    tile_distinct[t] = (uint32_t)dist;
    atomicAdd(big_out, outc);
  }
  __syncthreads();
}

// Persistent: workgroups take big tiles from a counter until none is left;
// item it of the work is big tile list[it] (an index into big_list /
// big_off), for it < *n_items.
template <int KW, bool kStream, bool kW>
__global__ void __launch_bounds__(kSortThreads)
k_big_tiles(KeyCfg kc, const Tile* __restrict__ tiles, const uint32_t* __restrict__ big_list,
            const uint64_t* __restrict__ big_off, const uint32_t* __restrict__ list,
            const uint32_t* n_items, uint32_t* next, uint64_t* keys, uint64_t* tmp,
            uint32_t* counts, uint32_t* tmpw, uint32_t* tile_out, uint32_t* tile_distinct,
            unsigned long long* big_out) {
  __shared__ uint32_t item;
  const uint32_t nb = *n_items;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(next, 1u);
    __syncthreads();
    const uint32_t it = item;
    __syncthreads();
    if (it >= nb) return;
    const uint32_t j = list[it];
    big_tile<KW, kStream, kW>(kc, tiles, big_list[j], big_off[j], keys, tmp, counts, tmpw,
                              tile_out, tile_distinct, big_out);
  }
}

// Big tiles of 64-bit keys, first pass: each is streamed through the LDS
// hash table (stream_count_hash); those with more distinct keys than the
// table takes are listed in fail_list for k_big_tiles.  A kernel of its own,
// so that its registers allow two workgroups per compute unit (the kernel
// that does both allows one).
template <bool kW>
__global__ void __launch_bounds__(kSortThreads)
k_big_stream(KeyCfg kc, const Tile* __restrict__ tiles, const uint32_t* __restrict__ big_list,
             const uint32_t* __restrict__ order, const uint32_t* n_big, uint32_t* next,
             uint64_t* keys, uint32_t* counts, uint32_t* tile_out, uint32_t* tile_distinct,
             unsigned long long* big_out, uint32_t* fail_list, uint32_t* n_fail) {
  __shared__ SortShared<1> S;
  __shared__ uint32_t item, claims;
  const uint32_t nb = *n_big;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(next, 1u);
    __syncthreads();
    const uint32_t it = item;
    __syncthreads();
    if (it >= nb) return;
    const uint32_t j = order[it], t = big_list[j];
    const Tile T = tiles[t];
    uint32_t d, kept;
    const bool ok = stream_count_hash<kW>(keys + T.begin, counts + T.begin, T.size,
                                          keys + T.begin, counts + T.begin, kc.cutoff_min,
                                          kc.cutoff_max, S, &claims, &d, &kept);
    if (threadIdx.x == 0) {
      if (ok) {
        tile_out[t] = kept;
        tile_distinct[t] = d;
        atomicAdd(big_out, (unsigned long long)kept);
      } else {
        fail_list[atomicAdd(n_fail, 1u)] = j;
      }
    }
    __syncthreads();  // the table is set up again for the next tile
  }
}

// The order in which the big-tile workgroups take the big tiles: largest
// first (a counting sort on the size in quarter octaves), so that the
// longest tiles start at once and the kernel does not end waiting on one
// big tile taken last.
constexpr uint32_t kSizeClasses = 128;
__device__ __forceinline__ uint32_t size_class(uint32_t size) {
  const uint32_t l = 31u - __clz(size | 4u);          // floor(log2), at least 2
  const uint32_t q = (size >> (l - 2)) & 3u;           // next two bits
  return kSizeClasses - 1u - min(4u * l + q, kSizeClasses - 1u);  // largest -> 0
}
// big_size[i] = size of big tile i (written beside big_list, so the reads
// here are sequential).
__global__ void __launch_bounds__(1024)
k_order_big(const uint32_t* __restrict__ big_size, const uint32_t* n_big, uint32_t* order) {
  __shared__ uint32_t cnt[kSizeClasses], tmp[16];
  const uint32_t nb = *n_big, tid = threadIdx.x;
  for (uint32_t i = tid; i < kSizeClasses; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < nb; i += blockDim.x) atomicAdd(&cnt[size_class(big_size[i])], 1u);
  __syncthreads();
  block_exclusive_scan(cnt, kSizeClasses, tmp);
  for (uint32_t i = tid; i < nb; i += blockDim.x)
    order[atomicAdd(&cnt[size_class(big_size[i])], 1u)] = i;
}

// ---------------------------------------------------------------- scans
constexpr uint32_t kScanChunk = 4096;  // elements per block (256 threads x 16)

__global__ void __launch_bounds__(256)
k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n, uint64_t* bsum) {
  __shared__ uint64_t red[4];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk;
  uint64_t s = 0;
  for (uint32_t i = threadIdx.x; i < kScanChunk; i += 256)
    if (b0 + i < n) s += in[b0 + i];
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one workgroup: exclusive scan of bsum[0..nb) in place, total to out[n]
__global__ void __launch_bounds__(256)
k_scan_bsum(uint64_t* bsum, uint64_t nb, uint64_t* out, uint64_t n) {
  __shared__ uint64_t wsum[4];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (uint64_t c0 = 0; c0 < nb; c0 += 256) {
    const uint64_t i = c0 + threadIdx.x;
    const uint64_t v = i < nb ? bsum[i] : 0;
    uint64_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
      uint64_t y = __shfl_up(x, d, 64);
      if (lane >= (uint32_t)d) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint64_t off = carry;
    for (uint32_t w = 0; w < wid; ++w) off += wsum[w];
    if (i < nb) bsum[i] = off + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ void __launch_bounds__(256)
k_scan_apply(const uint32_t* __restrict__ in, uint64_t n, const uint64_t* __restrict__ bsum,
             uint64_t* out) {
  __shared__ uint64_t wsum[4];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * 16;
  uint32_t v[16];
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    v[q] = (b0 + q < n) ? in[b0 + q] : 0u;
    s += v[q];
  }
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t x = s;
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  uint64_t run = bsum[blockIdx.x] + x - s;
  for (uint32_t w = 0; w < wid; ++w) run += wsum[w];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (b0 + q < n) out[b0 + q] = run;
    run += v[q];
  }
}

// ---------------------------------------------------------------- gather
// Counts are stored saturated at cmax (counter saturation; the cutoffs were
// applied to the exact counts before).
// One wavefront per tile, four tiles per workgroup (a tile keeps a few
// dozen entries: a workgroup per tile spent the kernel dispatching them).
template <int KW>
__global__ void __launch_bounds__(256)
k_gather(const Tile* __restrict__ tiles, const uint64_t* __restrict__ tile_off, uint64_t n_tiles,
         const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counts,
         uint64_t* out_keys, uint32_t* out_counts, uint32_t cmax) {
  const uint64_t t = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (t >= n_tiles) return;
  const uint64_t o = tile_off[t], m = tile_off[t + 1] - o;
  if (m == 0) return;
  const uint64_t b = tiles[t].begin;
  // 8-byte words: the output may be a caller's buffer with 8-byte alignment
  for (uint64_t i = lane; i < m * KW; i += 64) out_keys[o * KW + i] = keys[b * KW + i];
  for (uint64_t i = lane; i < m; i += 64) out_counts[o + i] = min(counts[b + i], cmax);
}

// ------------------------------------------------- global ascending order
// The table in ascending key order over all bins, instead of bin-major: the
// bin-major table is partitioned by the top bits of its keys (segments) into
// a scratch copy, consecutive segments are packed into groups of about
// CAP / 2 entries, and every group is put in order, back into the table, in
// LDS by the tile sort's ordering of kept keys (the keys are distinct, so
// nothing is counted).  A group above CAP
// entries (one segment of more than CAP / 2 keys that share their top bits)
// is merge sorted through HBM by its workgroup.

// Segment runs of the table in bin order (ascending inside each bin, so
// entries of a segment are adjacent within a bin): each thread takes
// kRunChunk consecutive entries and handles each of its runs with one
// atomic.  kScatter = false: entries per segment into seg_cnt; true: the run
// is copied to its segment at a slot claimed from the segment's cursor
// (seg_cnt, zeroed after the scan).
constexpr uint32_t kRunChunk = 16;
template <int KW, bool kScatter>
__global__ void __launch_bounds__(256)
k_seg_runs(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counts, uint64_t n,
           uint32_t shift, uint32_t* seg_cnt, const uint64_t* __restrict__ seg_start,
           uint64_t* xk, uint32_t* xc) {
  typedef typename KeyOf<KW>::T K;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kRunChunk;
  for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRunChunk; i0 < n;
       i0 += stride) {
    const uint64_t i1 = min(n, i0 + kRunChunk);
    uint64_t run = i0;
    uint32_t sg = (uint32_t)(load_key(keys, i0, (K*)nullptr) >> shift);
    for (uint64_t q = i0 + 1; q <= i1; ++q) {
      const uint32_t s2 = q < i1 ? (uint32_t)(load_key(keys, q, (K*)nullptr) >> shift) : ~0u;
      if (s2 == sg) continue;
      if (!kScatter) {
        atomicAdd(&seg_cnt[sg], (uint32_t)(q - run));
      } else {
        const uint64_t o = seg_start[sg] + atomicAdd(&seg_cnt[sg], (uint32_t)(q - run));
        for (uint64_t e = run; e < q; ++e) {
          store_key(xk, o + (e - run), load_key(keys, e, (K*)nullptr));
          xc[o + (e - run)] = counts[e];
        }
      }
      run = q;
      sg = s2;
    }
  }
}

// lo[g] = first segment start at or above g * G (lo[n_groups] = total);
// seg_start holds nseg + 1 entries, the last one the total.
__global__ void k_group_lo(const uint64_t* __restrict__ seg_start, uint64_t nseg, uint64_t G,
                           uint64_t n_groups, uint64_t* lo) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nseg) return;
  const uint64_t st = seg_start[s];
  // groups g with seg_start[s - 1] < g * G <= seg_start[s]
  const uint64_t g0 = s == 0 ? 0 : seg_start[s - 1] / G + 1;
  const uint64_t g1 = s == nseg ? n_groups : st / G;
  for (uint64_t g = g0; g <= g1; ++g) lo[g] = st;
}

// Entries [0, n) (n <= CAP, distinct keys) of xk / xc, in key order, to
// tk / tc.  All threads call it.
template <int KW>
__device__ void order_group(const uint64_t* xk, const uint32_t* xc, uint32_t n, uint64_t* tk,
                            uint32_t* tc, SortShared<KW>& S) {
  typedef typename KeyOf<KW>::T K;
  constexpr uint32_t ITEMS = SortCfg<KW>::ITEMS;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  K key[ITEMS];
  uint32_t cnt[ITEMS];
  K a = ~K(0), o = 0;
  uint32_t mine = 0;
#pragma unroll
  for (uint32_t m = 0; m < ITEMS; ++m) {
    const uint32_t i = m * nt + tid;
    cnt[m] = 0;
    if (i < n) {
      key[m] = load_key(xk, i, (K*)nullptr);
      cnt[m] = xc[i];  // a kept count is at least 1
      a &= key[m];
      o |= key[m];
      ++mine;
    }
  }
  uint32_t total;
  const uint32_t kbase = block_scan_one(mine, S.tmp, total);
  if (n == 1) {
    if (tid == 0) {
      store_key(tk, 0, key[0]);
      tc[0] = cnt[0];
    }
    __syncthreads();
    return;
  }
  block_and_or<K>(a, o, S.red);
  order_kept<KW>(key, cnt, kbase, n, a ^ o, tk, tc, S.A, S.H, S.tmp);
}

// Number of keys of src[b0, b1) below x (src ascending, distinct keys).
template <class K>
__device__ __forceinline__ uint64_t rank_in(const uint64_t* src, uint64_t b0, uint64_t b1,
                                            const K& x) {
  while (b0 < b1) {
    const uint64_t mid = (b0 + b1) / 2;
    if (load_key(src, mid, (K*)nullptr) < x) b0 = mid + 1;
    else b1 = mid;
  }
  return b0;
}

template <int KW>
__global__ void __launch_bounds__(kSortThreads)
k_group_sort(const uint64_t* __restrict__ lo, uint64_t* xk, uint32_t* xc, uint64_t* tk,
             uint32_t* tc) {
  typedef typename KeyOf<KW>::T K;
  constexpr uint32_t CAP = SortCfg<KW>::CAP;
  __shared__ SortShared<KW> S;
  const uint64_t g0 = lo[blockIdx.x], n = lo[blockIdx.x + 1] - g0;
  if (n == 0) return;
  xk += g0 * KW;
  xc += g0;
  tk += g0 * KW;
  tc += g0;
  if (n <= CAP) {
    order_group<KW>(xk, xc, (uint32_t)n, tk, tc, S);
    return;
  }
  // a group above CAP: chunks of CAP in order into t, then merge rounds
  // between t and x (a key's place in a merged pair is its place in its run
  // plus the number of keys of the other run below it)
  for (uint64_t c0 = 0; c0 < n; c0 += CAP)
    order_group<KW>(xk + c0 * KW, xc + c0, (uint32_t)min<uint64_t>(CAP, n - c0), tk + c0 * KW,
                    tc + c0, S);
  __threadfence();
  __syncthreads();
  uint64_t* sk = tk;
  uint32_t* sc = tc;
  uint64_t* dk = xk;
  uint32_t* dc = xc;
  for (uint64_t w = CAP; w < n; w *= 2) {
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint64_t p0 = i / (2 * w) * (2 * w), a1 = min(p0 + w, n), b1 = min(p0 + 2 * w, n);
      const K x = load_key(sk, i, (K*)nullptr);
      const uint64_t pos = i < a1 ? i + (rank_in(sk, a1, b1, x) - a1)
                                  : i - w + (rank_in(sk, p0, a1, x) - p0);
      store_key(dk, pos, x);
      dc[pos] = sc[i];
    }
    __threadfence();
    __syncthreads();
    uint64_t* t1 = sk;
    sk = dk;
    dk = t1;
    uint32_t* t2 = sc;
    sc = dc;
    dc = t2;
  }
  if (sk != tk) {
    for (uint64_t i = threadIdx.x; i < n * KW; i += blockDim.x) tk[i] = sk[i];
    for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) tc[i] = sc[i];
  }
}

}  // namespace

// Workgroups of kSortThreads that are resident at once on the current
// device: compute units x blocks per unit (by occupancy), cached per
// (kernel slot, device).
static int resident_blocks(const void* kernel, int slot) {
  constexpr int kSlots = 10, kDevs = 16;
  static std::atomic<int> cache[kSlots][kDevs];
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= kDevs) dev = 0;
  int v = cache[slot][dev].load(std::memory_order_relaxed);
  if (v) return v;
  int cus = 0, per_cu = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kSortThreads, 0);
  v = std::max(1, cus) * std::max(1, per_cu);
  cache[slot][dev].store(v, std::memory_order_relaxed);
  return v;
}

hipError_t launch_tile_sort(hipStream_t s, const KeyCfg& kc, const Tile* tiles,
                            uint64_t n_tiles, uint64_t* keys, uint32_t* out_counts,
                            uint32_t* tile_out, uint32_t* big_list, uint64_t* big_off,
                            uint32_t* n_big, unsigned long long* big_total,
                            uint32_t* tile_distinct, uint32_t* big_size, bool weighted) {
  if (n_tiles == 0) return hipSuccess;
  if (weighted && kc.key_words != 1) return hipErrorInvalidValue;
  // persistent grid: exactly the workgroups that are resident at once
  const void* kern = kc.key_words == 2 ? (const void*)k_tile_hash2
                     : weighted        ? (const void*)k_tile_sort<1, true>
                                       : (const void*)k_tile_sort<1, false>;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(
      n_tiles, (uint64_t)resident_blocks(kern, kc.key_words == 2 ? 1 : weighted ? 6 : 0));
  if (kc.key_words == 2)
    hipLaunchKernelGGL(k_tile_hash2, dim3(grid), dim3(kSortThreads), 0, s, kc,
                       tiles, n_tiles, keys, out_counts, tile_out, big_list, big_off, n_big, big_total,
                       tile_distinct, big_size);
  else if (weighted)
    hipLaunchKernelGGL((k_tile_sort<1, true>), dim3(grid), dim3(kSortThreads), 0, s, kc,
                       tiles, n_tiles, keys, out_counts, tile_out, big_list, big_off, n_big, big_total,
                       tile_distinct, big_size);
  else
    hipLaunchKernelGGL((k_tile_sort<1, false>), dim3(grid), dim3(kSortThreads), 0, s, kc,
                       tiles, n_tiles, keys, out_counts, tile_out, big_list, big_off, n_big, big_total,
                       tile_distinct, big_size);
  return hipGetLastError();
}

// The big-tile kernels of 64-bit keys, with or without weights.
template <bool kW>
static void big_tiles_64(hipStream_t s, const KeyCfg& kc, const Tile* tiles,
                         const uint32_t* big_list, const uint64_t* big_off, uint32_t* order,
                         uint32_t* fail_list, const uint32_t* n_big, uint32_t* next,
                         uint32_t* n_fail, uint32_t* fail_next, uint64_t max_big,
                         bool stream_first, uint64_t* keys, uint64_t* tmp, uint32_t* out_counts,
                         uint32_t* tmpw, uint32_t* tile_out, uint32_t* tile_distinct,
                         unsigned long long* big_out) {
  if (!stream_first) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(
        max_big, (uint64_t)resident_blocks((const void*)k_big_tiles<1, true, kW>, kW ? 7 : 5));
    hipLaunchKernelGGL((k_big_tiles<1, true, kW>), dim3(grid), dim3(kSortThreads), 0, s, kc,
                       tiles, big_list, big_off, order, n_big, next, keys, tmp, out_counts, tmpw,
                       tile_out, tile_distinct, big_out);
    return;
  }
  const uint32_t gs = (uint32_t)std::min<uint64_t>(
      max_big, (uint64_t)resident_blocks((const void*)k_big_stream<kW>, kW ? 8 : 4));
  hipLaunchKernelGGL(k_big_stream<kW>, dim3(gs), dim3(kSortThreads), 0, s, kc, tiles, big_list,
                     order, n_big, next, keys, out_counts, tile_out, tile_distinct, big_out,
                     fail_list, n_fail);
  const uint32_t grid = (uint32_t)std::min<uint64_t>(
      max_big, (uint64_t)resident_blocks((const void*)k_big_tiles<1, false, kW>, kW ? 9 : 2));
  hipLaunchKernelGGL((k_big_tiles<1, false, kW>), dim3(grid), dim3(kSortThreads), 0, s, kc,
                     tiles, big_list, big_off, fail_list, n_fail, fail_next, keys, tmp,
                     out_counts, tmpw, tile_out, tile_distinct, big_out);
}

hipError_t launch_big_tiles(hipStream_t s, const KeyCfg& kc, const Tile* tiles,
                            const uint32_t* big_list, const uint64_t* big_off,
                            const uint32_t* big_size, uint32_t* order,
                            uint32_t* fail_list, const uint32_t* n_big, uint32_t* next,
                            uint32_t* n_fail, uint32_t* fail_next, uint64_t max_big,
                            bool stream_first, uint64_t* keys, uint64_t* tmp,
                            uint32_t* out_counts, uint32_t* tmpw, uint32_t* tile_out,
                            uint32_t* tile_distinct, unsigned long long* big_out) {
  if (max_big == 0) return hipSuccess;
  if (tmpw && kc.key_words != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_order_big, dim3(1), dim3(1024), 0, s, big_size, n_big, order);
  if (kc.key_words == 1 && tmpw) {
    big_tiles_64<true>(s, kc, tiles, big_list, big_off, order, fail_list, n_big, next, n_fail,
                       fail_next, max_big, stream_first, keys, tmp, out_counts, tmpw, tile_out,
                       tile_distinct, big_out);
  } else if (kc.key_words == 1) {
    big_tiles_64<false>(s, kc, tiles, big_list, big_off, order, fail_list, n_big, next, n_fail,
                        fail_next, max_big, stream_first, keys, tmp, out_counts, nullptr,
                        tile_out, tile_distinct, big_out);
  } else {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(
        max_big, (uint64_t)resident_blocks((const void*)k_big_tiles<2, false, false>, 3));
    hipLaunchKernelGGL((k_big_tiles<2, false, false>), dim3(grid), dim3(kSortThreads), 0, s, kc,
                       tiles, big_list, big_off, order, n_big, next, keys, tmp, out_counts,
                       nullptr, tile_out, tile_distinct, big_out);
  }
  return hipGetLastError();
}

uint64_t scan_tmp_words(uint64_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

hipError_t launch_scan_u32(hipStream_t s, const uint32_t* in, uint64_t n, uint64_t* out,
                           uint64_t* block_tmp) {
  const uint64_t nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb == 0) {
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(256), 0, s, block_tmp, (uint64_t)0, out, n);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(256), 0, s, in, n, block_tmp);
  hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(256), 0, s, block_tmp, nb, out, n);
  hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)nb), dim3(256), 0, s, in, n, block_tmp, out);
  return hipGetLastError();
}

hipError_t launch_gather(hipStream_t s, const KeyCfg& kc, const Tile* tiles, uint64_t n_tiles,
                         const uint64_t* tile_off, const uint64_t* keys,
                         const uint32_t* counts, uint64_t* out_keys, uint32_t* out_counts) {
  if (n_tiles == 0) return hipSuccess;
  const dim3 g((uint32_t)((n_tiles + 3) / 4));
  if (kc.key_words == 1)
    hipLaunchKernelGGL(k_gather<1>, g, dim3(256), 0, s, tiles, tile_off, n_tiles, keys, counts,
                       out_keys, out_counts, kc.counter_max);
  else
    hipLaunchKernelGGL(k_gather<2>, g, dim3(256), 0, s, tiles, tile_off, n_tiles, keys, counts,
                       out_keys, out_counts, kc.counter_max);
  return hipGetLastError();
}

AscPlan plan_ascending(uint64_t n_out, uint32_t k, uint32_t key_words) {
  AscPlan ap;
  const uint64_t cap = key_words == 1 ? kTileCap1 : kTileCap2;
  ap.group = cap / 2;
  // segments of about cap / 16 entries on average
  uint32_t b = 1;
  while (b < kMaxSegBits && ((n_out * 16) >> b) > cap) ++b;
  ap.seg_bits = std::min<uint32_t>(b, 2 * k);
  ap.n_groups = (n_out + ap.group - 1) / ap.group;
  return ap;
}

hipError_t launch_ascending(hipStream_t s, const KeyCfg& kc, uint64_t n_out, const AscPlan& ap,
                            uint32_t* seg_cnt, uint64_t* seg_start, uint64_t* scan_tmp,
                            uint64_t* lo, uint64_t* xk, uint32_t* xc, uint64_t* table_keys,
                            uint32_t* table_counts) {
  if (n_out == 0 || ap.n_groups == 0) return hipSuccess;
  const uint64_t nseg = 1ull << ap.seg_bits;
  const uint32_t shift = 2 * kc.k - ap.seg_bits;
  const uint64_t chunks = (n_out + kRunChunk - 1) / kRunChunk;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((chunks + 255) / 256, 65535);
  hipError_t e = hipMemsetAsync(seg_cnt, 0, nseg * 4, s);
  if (e != hipSuccess) return e;
  const bool one = kc.key_words == 1;
  if (one)
    hipLaunchKernelGGL((k_seg_runs<1, false>), dim3(grid), dim3(256), 0, s, table_keys,
                       table_counts, n_out, shift, seg_cnt, seg_start, xk, xc);
  else
    hipLaunchKernelGGL((k_seg_runs<2, false>), dim3(grid), dim3(256), 0, s, table_keys,
                       table_counts, n_out, shift, seg_cnt, seg_start, xk, xc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_scan_u32(s, seg_cnt, nseg, seg_start, scan_tmp)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_lo, dim3((uint32_t)((nseg + 1 + 255) / 256)), dim3(256), 0, s,
                     seg_start, nseg, ap.group, ap.n_groups, lo);
  if ((e = hipMemsetAsync(seg_cnt, 0, nseg * 4, s)) != hipSuccess) return e;
  if (one)
    hipLaunchKernelGGL((k_seg_runs<1, true>), dim3(grid), dim3(256), 0, s, table_keys,
                       table_counts, n_out, shift, seg_cnt, seg_start, xk, xc);
  else
    hipLaunchKernelGGL((k_seg_runs<2, true>), dim3(grid), dim3(256), 0, s, table_keys,
                       table_counts, n_out, shift, seg_cnt, seg_start, xk, xc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (one)
    hipLaunchKernelGGL(k_group_sort<1>, dim3((uint32_t)ap.n_groups), dim3(kSortThreads), 0, s,
                       lo, xk, xc, table_keys, table_counts);
  else
    hipLaunchKernelGGL(k_group_sort<2>, dim3((uint32_t)ap.n_groups), dim3(kSortThreads), 0, s,
                       lo, xk, xc, table_keys, table_counts);
  return hipGetLastError();
}

}  // namespace kmc

namespace kmc {
namespace {
__global__ void k_bin_offsets(const uint64_t* __restrict__ tile_off,
                              const uint64_t* __restrict__ tile_base, uint32_t n_bins,
                              uint64_t* out) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= n_bins) out[b] = tile_off[tile_base[b]];
}
}  // namespace

hipError_t launch_bin_offsets(hipStream_t s, const uint64_t* tile_off, const uint64_t* tile_base,
                              uint32_t n_bins, uint64_t* out) {
  hipLaunchKernelGGL(k_bin_offsets, dim3((n_bins + 256) / 256), dim3(256), 0, s, tile_off,
                     tile_base, n_bins, out);
  return hipGetLastError();
}
}  // namespace kmc
