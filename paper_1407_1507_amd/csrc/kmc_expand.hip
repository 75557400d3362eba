// Sorting phase, first half: per-bin extraction of canonical k-mers from the
// super k-mer records and their partition into tiles small enough to be
// sorted inside one workgroup's LDS.
//
// Method (KMC 2, Methods, "Sketch of the algorithm"): each bin is read, every
// k-mer of every super k-mer is extracted in canonical form (the smaller of
// the k-mer and its reverse complement, "Minimizers of k-mers") and the keys
// are radix sorted.  Here the most significant digit pass of that radix sort
// runs through HBM: each bin's keys are split by their top `fine_bits` bits
// into fine ranges, consecutive fine ranges are packed into tiles of at most
// `tile_limit` keys, and every key is written to its tile.  A tile is thus a
// contiguous key range of one bin, and tiles of a bin are in key order.
//
// Record layout (written by the split kernels): forward key of the first
// k-mer, then the remaining symbols left aligned with the k-mer count in the
// low 8 bits.  Keys are rolled forward and reverse-complement at once.
#include <type_traits>

#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

namespace {

template <int KW> struct Rec;
template <> struct Rec<1> {
  uint64_t F, R, T;
  uint32_t n;
  bool canon;  // canonical keys; else the forward k-mer itself
  __device__ void load(const uint64_t* r, uint32_t k, bool canonical = true) {
    F = r[0];
    T = r[1];
    n = (uint32_t)(T & 0xFFu);
    R = revcomp64(F, k);
    canon = canonical;
  }
  __device__ uint64_t key() const { return canon && R < F ? R : F; }
  __device__ void step(uint32_t k, uint64_t kmask) {
    const uint32_t c = (uint32_t)(T >> 62);
    T <<= 2;
    F = ((F << 2) | c) & kmask;
    R = (R >> 2) | ((uint64_t)(3u - c) << (2 * k - 2));
  }
};
// 128-bit keys (33 <= k <= 64) as high and low words: every shift by an
// amount that depends on k stays inside one word (the reverse complement's
// new symbol enters the high word at bit 2k - 66), where a 128-bit shift by a
// run-time amount costs selects between the words at each step.
template <> struct Rec<2> {
  uint64_t Fh, Fl, Rh, Rl, Th, Tl;
  uint32_t n;
  bool canon;
  __device__ void load(const uint64_t* r, uint32_t k, bool canonical = true) {
    Fh = r[0];
    Fl = r[1];
    Th = r[2];
    Tl = r[3];
    n = (uint32_t)(Tl & 0xFFu);
    const u128 R = revcomp128(((u128)Fh << 64) | Fl, k);
    Rh = (uint64_t)(R >> 64);
    Rl = (uint64_t)R;
    canon = canonical;
  }
  // the canonical key is the reverse complement
  __device__ bool rev() const { return canon && (Rh < Fh || (Rh == Fh && Rl < Fl)); }
  __device__ u128 key() const {
    const bool r = rev();
    return ((u128)(r ? Rh : Fh) << 64) | (r ? Rl : Fl);
  }
  __device__ void step(uint32_t k, u128 kmask) {
    const uint64_t c = Th >> 62;
    Th = (Th << 2) | (Tl >> 62);
    Tl <<= 2;
    Fh = ((Fh << 2) | (Fl >> 62)) & (uint64_t)(kmask >> 64);
    Fl = (Fl << 2) | c;
    Rl = (Rl >> 2) | (Rh << 62);
    Rh = (Rh >> 2) | ((3 - c) << (2 * k - 66));
  }
};

// top `bits` bits of a 2k-bit key
__device__ __forceinline__ uint32_t top_bits(uint64_t key, uint32_t k, uint32_t bits) {
  return (uint32_t)(key >> (2 * k - bits));
}
__device__ __forceinline__ uint32_t top_bits(u128 key, uint32_t k, uint32_t bits) {
  return (uint32_t)(key >> (2 * k - bits));
}
// the same for a 128-bit key as words, sh = 2k - bits (>= 1)
__device__ __forceinline__ uint32_t top_bits2(uint64_t h, uint64_t l, uint32_t sh) {
  return sh >= 64 ? (uint32_t)(h >> (sh - 64)) : (uint32_t)((h << (64 - sh)) | (l >> sh));
}

// The top b bits of a canonical key, min(F, R) >> (2k - b), are min(F >> (2k
// - b), R >> (2k - b)): a shift keeps the order.  So a walk that needs only
// those bits keeps the forward key and just the top bits of the reverse
// complement, which roll on their own: R' = (R >> 2) | (3 - c) << (2k - 2)
// gives top(R') = (top(R) >> 2) | (3 - c) << (b - 2) (b >= 2).
template <int KW> struct RecTop;
template <> struct RecTop<1> {
  uint64_t F, T;
  uint32_t rt, n;
  bool canon;
  __device__ void load(const uint64_t* r, uint32_t k, uint32_t sh, bool canonical) {
    Rec<1> full;
    full.load(r, k);
    F = full.F;
    T = full.T;
    n = full.n;
    rt = (uint32_t)(full.R >> sh);
    canon = canonical;
  }
  __device__ uint32_t top(uint32_t sh) const {
    const uint32_t f = (uint32_t)(F >> sh);
    return canon ? min(f, rt) : f;
  }
  __device__ void step(uint64_t kmask, uint32_t bits) {
    const uint32_t c = (uint32_t)(T >> 62);
    T <<= 2;
    F = ((F << 2) | c) & kmask;
    rt = (rt >> 2) | ((3u - c) << (bits - 2));
  }
};
template <> struct RecTop<2> {
  u128 F, T;
  uint32_t rt, n;
  bool canon;
  __device__ void load(const uint64_t* r, uint32_t k, uint32_t sh, bool canonical) {
    Rec<2> full;
    full.load(r, k);
    F = ((u128)full.Fh << 64) | full.Fl;
    T = ((u128)full.Th << 64) | full.Tl;
    n = full.n;
    rt = top_bits2(full.Rh, full.Rl, sh);
    canon = canonical;
  }
  __device__ uint32_t top(uint32_t sh) const {
    const uint32_t f = (uint32_t)(F >> sh);
    return canon ? min(f, rt) : f;
  }
  __device__ void step(u128 kmask, uint32_t bits) {
    const uint32_t c = (uint32_t)(T >> 126);
    T <<= 2;
    F = ((F << 2) | (u128)c) & kmask;
    rt = (rt >> 2) | ((3u - c) << (bits - 2));
  }
};

// --------------------------------------------------------------- (k,x)-mers
// Methods, "(k,x)-mers", and Fig. 2: a super k-mer is cut into the fewest
// (k + x')-mers (x' <= x) whose k-mers are all canonical in the same
// direction: walking its k-mers in order, a piece grows while the next k-mer
// has the direction of the piece's first (forward when it is not larger than
// its reverse complement, else reverse) and the piece holds at most x + 1
// k-mers.  A forward piece is stored as read, a reverse piece as its reverse
// complement, so every k-mer inside it is canonical.  Key (64 bits, k + x
// <= 31): x' in the top two bits, the (k + x')-mer left-aligned below, the
// rest zero; keys thus sort by x' first, then by sequence (the order of the
// figure: the k-mers, then the (k+1)-mers).
__device__ __forceinline__ uint64_t kx_key(uint64_t seq, uint32_t len, uint32_t xp) {
  return ((uint64_t)xp << 62) | (seq << (62 - 2 * len));
}
// f(key) for every (k,x)-mer of the staged record r (64-bit k-mers)
template <class F>
__device__ __forceinline__ void kx_pieces(const uint64_t* r, const KeyCfg& kc, F f) {
  Rec<1> rec;
  rec.load(r, kc.k, true);
  const uint64_t kmask = key_mask<uint64_t>(kc.k);
  uint64_t E = rec.F;  // the piece's symbols as read
  uint32_t len = 1;    // k-mers in the piece
  bool rev = rec.R < rec.F;
  auto emit = [&]() {
    const uint32_t xp = len - 1, L = kc.k + xp;
    f(kx_key(rev ? revcomp64(E, L) : E, L, xp));
  };
  for (uint32_t i = 1; i < rec.n; ++i) {
    const uint32_t c = (uint32_t)(rec.T >> 62);
    rec.step(kc.k, kmask);
    const bool ri = rec.R < rec.F;
    if (ri == rev && len <= kc.kx) {
      E = (E << 2) | c;
      ++len;
    } else {
      emit();
      E = rec.F;
      len = 1;
      rev = ri;
    }
  }
  emit();
}
// f(k-mer, weight) for the k-mers of a distinct (k,x)-mer record r (word 0
// its key, word 1 its count << 8 | k-mers)
template <class F>
__device__ __forceinline__ void kx_kmers(const uint64_t* r, const KeyCfg& kc, F f) {
  const uint64_t key = r[0];
  const uint32_t xp = (uint32_t)(key >> 62), L = kc.k + xp;
  const uint64_t E = (key & ((1ull << 62) - 1)) >> (62 - 2 * L);
  const uint32_t w = (uint32_t)(r[1] >> 8);
  const uint64_t kmask = key_mask<uint64_t>(kc.k);
  for (uint32_t j = 0; j <= xp; ++j) f((E >> (2 * (xp - j))) & kmask, w);
}

// ------------------------------------------------------------ round staging
// A super k-mer holds 1 .. w k-mers, so with one record per lane a wavefront
// runs as long as its longest record.  Each round of up to 256 records is
// therefore staged in LDS and ranked by k-mer count, longest first (a
// counting sort on the count byte): slot s of the round is the s-th longest
// record, and each wavefront walks records of similar length.
template <int KW>
struct RoundLds {
  uint64_t w[kExpandThreads * 2 * KW];  // the round's records, as stored
  uint32_t hist[64];                     // count buckets, then their offsets
  uint8_t perm[kExpandThreads];          // slot -> record of the round
};

// Stage records rp[0 .. nr) (nr <= blockDim.x = kExpandThreads); all threads
// call it.  On return slot t's record is L.w + L.perm[t] * 2 * KW.
template <int KW>
__device__ __forceinline__ void stage_round(const uint64_t* __restrict__ rp, uint32_t nr,
                                            RoundLds<KW>& L) {
  const uint32_t t = threadIdx.x;
  if (t < 64) L.hist[t] = 0;
  __syncthreads();  // the previous round's slots are done with w and perm
  uint32_t bucket = 0, rank = 0;
  if (t < nr) {
    const uint4* src = reinterpret_cast<const uint4*>(rp + (size_t)t * 2 * KW);
    uint4* dst = reinterpret_cast<uint4*>(L.w + (size_t)t * 2 * KW);
    uint4 last;
#pragma unroll
    for (int i = 0; i < KW; ++i) {
      last = src[i];
      dst[i] = last;
    }
    const uint32_t n = last.z & 0xFFu;  // count byte: low byte of the last word
    bucket = 63u - (n < 63u ? n : 63u);
    rank = atomicAdd(&L.hist[bucket], 1u);
  }
  __syncthreads();
  if (t < 64) {
    const uint32_t v = L.hist[t];
    uint32_t incl = v;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
      const uint32_t u = __shfl_up(incl, d, 64);
      if (t >= d) incl += u;
    }
    L.hist[t] = incl - v;
  }
  __syncthreads();
  if (t < nr) L.perm[L.hist[bucket] + rank] = (uint8_t)t;
  __syncthreads();
}

// Workgroups are dealt to the chip's 8 XCDs in turn (workgroup i to XCD
// i mod 8), each XCD with its own L2.  xcd_task maps workgroup i so that XCD
// x takes the contiguous tasks [x * per, (x + 1) * per): tasks are ordered by
// bin and a bin's tiles take keys from that bin's tasks only, so the partial
// lines that neighbouring tasks write into a tile meet in one L2.  The grid is
// 8 * per workgroups; indices at or past n_tasks have no task.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_task(uint32_t i, uint32_t per) {
  return (i % kXcds) * per + i / kXcds;
}

// --------------------------------------------------------------- fine hist
// One workgroup per task (a run of records of one bin); the task's keys are
// counted per fine range in LDS, then added to the bin's global histogram.
__global__ void __launch_bounds__(256)
k_task_bins(const uint64_t* __restrict__ pre_a, uint16_t* bin_a, const uint64_t* __restrict__ pre_b,
            const uint64_t* __restrict__ rec_base, const uint64_t* __restrict__ rec_end,
            uint32_t per_b, ExpandTask* desc_b) {
  const uint32_t b = blockIdx.x;
  for (uint64_t t = pre_a[b] + threadIdx.x; t < pre_a[b + 1]; t += blockDim.x) bin_a[t] = (uint16_t)b;
  for (uint64_t t = pre_b[b] + threadIdx.x; t < pre_b[b + 1]; t += blockDim.x) {
    ExpandTask k;
    k.bin = b;
    k.rec_begin = rec_base[b] + (t - pre_b[b]) * per_b;
    const uint64_t left = rec_end[b] - k.rec_begin;
    k.n_rec = left < per_b ? (uint32_t)left : per_b;
    desc_b[t] = k;
  }
}

// MODE: 0 the k-mers of the records; 1 their (k,x)-mers; 2 the k-mers of
// distinct (k,x)-mer records (KeyCfg::kx_pass; 1 and 2 with 64-bit keys).
template <int KW, int MODE>
__global__ void __launch_bounds__(kExpandThreads)
k_fine_hist(KeyCfg kc, TaskMap tm, const uint64_t* __restrict__ records, uint32_t* fine_hist) {
  typedef typename KeyOf<KW>::T K;
  extern __shared__ __attribute__((aligned(16))) uint64_t lds64[];
  RoundLds<KW>& L = *reinterpret_cast<RoundLds<KW>*>(lds64);
  uint32_t* fh = reinterpret_cast<uint32_t*>(&L + 1);
  const uint32_t nf = 1u << kc.fine_bits;
  for (uint32_t i = threadIdx.x; i < nf; i += blockDim.x) fh[i] = 0;
  const ExpandTask tk = tm.get(blockIdx.x);
  const K kmask = key_mask<K>(kc.k);
  for (uint32_t r0 = 0; r0 < tk.n_rec; r0 += kExpandThreads) {
    const uint32_t nr = min(tk.n_rec - r0, (uint32_t)kExpandThreads);
    stage_round<KW>(records + (tk.rec_begin + r0) * (2 * KW), nr, L);
    if constexpr (MODE == 1) {
      if (threadIdx.x < nr)
        kx_pieces(L.w + (uint32_t)L.perm[threadIdx.x] * 2, kc, [&](uint64_t key) {
          atomicAdd(&fh[(uint32_t)(key >> (64 - kc.fine_bits))], 1u);
        });
    } else if constexpr (MODE == 2) {
      if (threadIdx.x < nr)
        kx_kmers(L.w + (uint32_t)L.perm[threadIdx.x] * 2, kc, [&](uint64_t y, uint32_t) {
          atomicAdd(&fh[top_bits(y, kc.k, kc.fine_bits)], 1u);
        });
    } else if (threadIdx.x < nr && kc.fine_bits >= 2) {
      // only the top fine_bits bits of each key: see RecTop
      const uint32_t sh = 2 * kc.k - kc.fine_bits;
      RecTop<KW> rec;
      rec.load(L.w + (uint32_t)L.perm[threadIdx.x] * (2 * KW), kc.k, sh, kc.canonical != 0);
      for (uint32_t i = 0;; ++i) {
        atomicAdd(&fh[rec.top(sh)], 1u);
        if (i + 1 >= rec.n) break;
        rec.step(kmask, kc.fine_bits);
      }
    } else if (threadIdx.x < nr) {
      Rec<KW> rec;
      rec.load(L.w + (uint32_t)L.perm[threadIdx.x] * (2 * KW), kc.k, kc.canonical != 0);
      for (uint32_t i = 0;; ++i) {
        atomicAdd(&fh[top_bits(rec.key(), kc.k, kc.fine_bits)], 1u);
        if (i + 1 >= rec.n) break;
        rec.step(kc.k, kmask);
      }
    }
  }
  __syncthreads();
  uint32_t* gh = fine_hist + ((uint64_t)tk.bin << kc.fine_bits);
  for (uint32_t i = threadIdx.x; i < nf; i += blockDim.x)
    if (fh[i]) atomicAdd(&gh[i], fh[i]);
}

// -------------------------------------------------------------- plan tiles
// One workgroup per bin.  Consecutive fine ranges are packed greedily into
// tiles of at most tile_limit keys: a tile is closed when the next range would
// take it past the limit (a range larger than the limit is a tile of its own,
// a big tile, which with big_merge set also takes the following ranges while
// it holds at most big_merge keys).
// Two consecutive tiles then hold more than tile_limit keys together, so a bin
// of T keys needs at most 2 * ceil(T / tile_limit) + 1 tiles; slots beyond
// the ones used stay empty (the tile array is zeroed beforehand).
//
// In parallel: for every range r, nxt[r] = the range that would start the next
// tile if a tile started at r (a binary search over the prefix sums); one
// thread then follows the chain from range 0 (one step per tile), and the
// tiles are written in parallel.
__global__ void __launch_bounds__(256)
k_plan_tiles(KeyCfg kc, const uint32_t* __restrict__ fine_hist, const uint64_t* __restrict__ key_base,
             const uint64_t* __restrict__ tile_base, uint16_t* tile_of_fine, Tile* tiles,
             unsigned long long* tile_cursor) {
  extern __shared__ uint32_t lds[];
  const uint32_t nf = 1u << kc.fine_bits;
  uint32_t* start = lds;                                          // nf + 1
  uint16_t* nxt = reinterpret_cast<uint16_t*>(start + nf + 1);    // nf (+1 spare)
  uint16_t* chain = nxt + nf + 2;                                 // tile starts, <= nf + 1
  uint32_t* tmp = reinterpret_cast<uint32_t*>(chain + nf + 2);    // scan tmp, tile count
  const uint32_t b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const uint32_t* h = fine_hist + ((uint64_t)b << kc.fine_bits);
  for (uint32_t i = tid; i < nf; i += nt) start[i] = h[i];
  __syncthreads();
  const uint32_t total = block_exclusive_scan(start, nf, tmp);
  if (tid == 0) start[nf] = total;
  __syncthreads();
  if (total == 0) return;  // empty bin: no tiles
  const uint32_t lim = kc.tile_limit;
  for (uint32_t r = tid; r < nf; r += nt) {
    const uint32_t s0 = start[r];
    // q1: the smallest q > r with start[q + 1] > s0 + lim (nf if none)
    uint32_t lo = r + 1, hi = nf;  // answer in [lo, hi]
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (start[mid + 1] > s0 + lim) hi = mid;
      else lo = mid + 1;
    }
    uint32_t q = lo;
    // a tile still empty at q1 takes range q1 too (a range over the limit)
    if (q < nf && start[q] == s0) ++q;
    if (kc.big_merge && start[min(q, nf)] - s0 > lim) {
      // a big tile: the following ranges too, while it holds at most
      // big_merge keys (q2: the smallest q2 >= q with start[q2 + 1] > s0 +
      // big_merge, nf if none)
      uint32_t lo2 = q, hi2 = nf;
      while (lo2 < hi2) {
        const uint32_t mid = (lo2 + hi2) >> 1;
        if (start[mid + 1] > s0 + kc.big_merge) hi2 = mid;
        else lo2 = mid + 1;
      }
      q = max(q, lo2);
    }
    nxt[r] = (uint16_t)min(q, nf);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t c = 0, t = 0;
    while (c < nf) {
      chain[t++] = (uint16_t)c;
      c = nxt[c];
    }
    chain[t] = (uint16_t)nf;
    tmp[0] = t;
  }
  __syncthreads();
  const uint32_t n_used = tmp[0];
  const uint64_t kb = key_base[b], tb = tile_base[b];
  uint16_t* tof = tile_of_fine + ((uint64_t)b << kc.fine_bits);
  for (uint32_t t = tid; t < n_used; t += nt) {
    const uint32_t r0 = chain[t], r1 = chain[t + 1];
    const uint32_t first = start[r0];
    tiles[tb + t] = Tile{kb + first, start[r1] - first, b};
    tile_cursor[tb + t] = kb + first;
    for (uint32_t r = r0; r < r1; ++r) tof[r] = (uint16_t)t;
  }
}

// ---------------------------------------------------------- expand scatter
// One workgroup per task (a run of records of one bin, staged a round of
// blockDim records at a time, one per lane).  Two walks over each record's
// k-mers: the first counts keys per tile in LDS; after one global
// reservation per (task, tile) the second walk writes every key straight to
// its slot, tile slot = reserved start + rank from an LDS counter.  A task's
// keys of one tile land in one contiguous range.  No barrier inside the
// walks.
// MODE as for k_fine_hist; with MODE 2 each key's weight goes to weights at
// the key's slot.
template <int KW, int MODE>
__global__ void __launch_bounds__(kExpandThreads)
k_expand_scatter(KeyCfg kc, TaskMap tm,
                 const uint64_t* __restrict__ records, const uint16_t* __restrict__ tile_of_fine,
                 const uint64_t* __restrict__ tile_base, const uint64_t* __restrict__ key_base,
                 uint32_t mt, uint32_t n_tasks, unsigned long long* tile_cursor,
                 uint64_t* keys, uint32_t* weights) {
  typedef typename KeyOf<KW>::T K;
  // a tile's reserved start: for 64-bit keys 32 bits relative to the bin's
  // first key (a bin holds fewer than 2^32), so the per-tile arrays take 8
  // bytes a tile and bins of thousands of tiles leave room for more
  // workgroups; 128-bit keys keep 64 bits (measured faster there)
  typedef typename std::conditional<KW == 1, uint32_t, uint64_t>::type Off;
  extern __shared__ __attribute__((aligned(16))) uint64_t lds64[];
  const uint32_t nf = 1u << kc.fine_bits;
  // layout: round records | delta Off[mt] | cnt u32[mt] | tof u16[nf]
  RoundLds<KW>& L = *reinterpret_cast<RoundLds<KW>*>(lds64);
  Off* delta = reinterpret_cast<Off*>(&L + 1);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(delta + mt);
  uint16_t* tof = reinterpret_cast<uint16_t*>(cnt + mt);

  // 128-bit keys by XCD (the 16-byte scatter otherwise writes back about
  // twice its bytes); 64-bit keys in launch order, which measured faster
  const uint32_t task =
      KW == 2 ? xcd_task(blockIdx.x, (n_tasks + kXcds - 1) / kXcds) : blockIdx.x;
  if (task >= n_tasks) return;
  const ExpandTask tk = tm.get(task);
  const uint16_t* gt = tile_of_fine + ((uint64_t)tk.bin << kc.fine_bits);
  for (uint32_t i = threadIdx.x; i < nf; i += blockDim.x) tof[i] = gt[i];
  const uint64_t tb = tile_base[tk.bin];
  const uint32_t nt = (uint32_t)(tile_base[tk.bin + 1] - tb);  // <= mt
  const uint64_t kb = KW == 1 ? key_base[tk.bin] : 0;
  for (uint32_t i = threadIdx.x; i < nt; i += blockDim.x) cnt[i] = 0;
  const K kmask = key_mask<K>(kc.k);
  const bool canon = kc.canonical != 0;
  // walk 1 over the slot's staged record: keys per tile
  auto count_walk = [&](const uint64_t* my) {
    if constexpr (MODE == 1) {
      kx_pieces(my, kc, [&](uint64_t key) {
        atomicAdd(&cnt[tof[(uint32_t)(key >> (64 - kc.fine_bits))]], 1u);
      });
      return;
    } else if constexpr (MODE == 2) {
      kx_kmers(my, kc, [&](uint64_t y, uint32_t) {
        atomicAdd(&cnt[tof[top_bits(y, kc.k, kc.fine_bits)]], 1u);
      });
      return;
    }
    if (kc.fine_bits >= 2) {
      // only the top fine_bits bits of each key: see RecTop
      const uint32_t sh = 2 * kc.k - kc.fine_bits;
      RecTop<KW> rec;
      rec.load(my, kc.k, sh, canon);
      for (uint32_t i = 0;; ++i) {
        atomicAdd(&cnt[tof[rec.top(sh)]], 1u);
        if (i + 1 >= rec.n) break;
        rec.step(kmask, kc.fine_bits);
      }
      return;
    }
    Rec<KW> rec;
    rec.load(my, kc.k, canon);
    for (uint32_t i = 0;; ++i) {
      atomicAdd(&cnt[tof[top_bits(rec.key(), kc.k, kc.fine_bits)]], 1u);
      if (i + 1 >= rec.n) break;
      rec.step(kc.k, kmask);
    }
  };
  // walk 2: the same keys again, each written to its tile
  auto write_walk = [&](const uint64_t* my) {
    if constexpr (MODE == 1) {
      kx_pieces(my, kc, [&](uint64_t key) {
        const uint32_t t = tof[(uint32_t)(key >> (64 - kc.fine_bits))];
        keys[kb + delta[t] + atomicAdd(&cnt[t], 1u)] = key;
      });
      return;
    } else if constexpr (MODE == 2) {
      kx_kmers(my, kc, [&](uint64_t y, uint32_t w) {
        const uint32_t t = tof[top_bits(y, kc.k, kc.fine_bits)];
        const uint64_t g = kb + delta[t] + atomicAdd(&cnt[t], 1u);
        keys[g] = y;
        weights[g] = w;
      });
      return;
    }
    Rec<KW> rec;
    rec.load(my, kc.k, canon);
    if constexpr (KW == 2) {
      const uint32_t sh = 2 * kc.k - kc.fine_bits;
      for (uint32_t i = 0;; ++i) {
        const bool r = rec.rev();
        const uint64_t h = r ? rec.Rh : rec.Fh, l = r ? rec.Rl : rec.Fl;
        const uint32_t t = tof[top_bits2(h, l, sh)];
        const uint64_t g = delta[t] + atomicAdd(&cnt[t], 1u);
        reinterpret_cast<ulonglong2*>(keys)[g] = make_ulonglong2(h, l);
        if (i + 1 >= rec.n) break;
        rec.step(kc.k, kmask);
      }
    } else {
      for (uint32_t i = 0;; ++i) {
        const K key = rec.key();
        const uint32_t t = tof[top_bits(key, kc.k, kc.fine_bits)];
        keys[kb + delta[t] + atomicAdd(&cnt[t], 1u)] = (uint64_t)key;
        if (i + 1 >= rec.n) break;
        rec.step(kc.k, kmask);
      }
    }
  };
  // reserve each tile's range; cnt then becomes the running slot
  auto reserve = [&]() {
    for (uint32_t i = threadIdx.x; i < nt; i += blockDim.x) {
      const uint32_t c = cnt[i];
      if (c) delta[i] = (Off)(atomicAdd(&tile_cursor[tb + i], (unsigned long long)c) - kb);
      cnt[i] = 0;
    }
  };
  const uint64_t* base = records + tk.rec_begin * (2 * KW);
  if (tk.n_rec <= kExpandThreads) {
    // one round: staged once, walked twice
    stage_round<KW>(base, tk.n_rec, L);
    const uint64_t* my = L.w + (uint32_t)L.perm[threadIdx.x] * (2 * KW);
    if (threadIdx.x < tk.n_rec) count_walk(my);
    __syncthreads();
    reserve();
    __syncthreads();
    if (threadIdx.x < tk.n_rec) write_walk(my);
    return;
  }
  // several rounds (longer runs of keys per tile): every round staged for
  // the counting walk, one reservation per tile, then staged again for the
  // writing walk
  for (uint32_t r0 = 0; r0 < tk.n_rec; r0 += kExpandThreads) {
    const uint32_t nr = min(tk.n_rec - r0, (uint32_t)kExpandThreads);
    stage_round<KW>(base + (uint64_t)r0 * (2 * KW), nr, L);
    if (threadIdx.x < nr) count_walk(L.w + (uint32_t)L.perm[threadIdx.x] * (2 * KW));
  }
  __syncthreads();
  reserve();
  __syncthreads();
  for (uint32_t r0 = 0; r0 < tk.n_rec; r0 += kExpandThreads) {
    const uint32_t nr = min(tk.n_rec - r0, (uint32_t)kExpandThreads);
    stage_round<KW>(base + (uint64_t)r0 * (2 * KW), nr, L);
    if (threadIdx.x < nr) write_walk(L.w + (uint32_t)L.perm[threadIdx.x] * (2 * KW));
  }
}

__global__ void __launch_bounds__(256)
k_kx_records(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counts, uint64_t n,
             uint64_t* records) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = keys[i];
  ulonglong2 r;
  r.x = key;
  r.y = ((uint64_t)counts[i] << 8) | ((key >> 62) + 1);
  reinterpret_cast<ulonglong2*>(records)[i] = r;
}

}  // namespace

hipError_t launch_kx_records(hipStream_t s, const uint64_t* keys, const uint32_t* counts,
                             uint64_t n, uint64_t* records) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kx_records, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, keys,
                     counts, n, records);
  return hipGetLastError();
}

static size_t round_lds(int kw) {
  return kw == 1 ? sizeof(RoundLds<1>) : sizeof(RoundLds<2>);
}
static size_t expand_lds(int kw, uint32_t mt, uint32_t nf) {
  return round_lds(kw) + (size_t)mt * (kw == 1 ? 8 : 12) + (size_t)nf * 2;
}

hipError_t launch_task_bins(hipStream_t s, uint32_t n_bins, const uint64_t* pre_a,
                            uint16_t* bin_a, const uint64_t* pre_b, const uint64_t* rec_base,
                            const uint64_t* rec_end, uint32_t per_b, ExpandTask* desc_b) {
  hipLaunchKernelGGL(k_task_bins, dim3(n_bins), dim3(256), 0, s, pre_a, bin_a, pre_b, rec_base,
                     rec_end, per_b, desc_b);
  return hipGetLastError();
}

hipError_t launch_fine_hist(hipStream_t s, const KeyCfg& kc, const TaskMap& tm,
                            uint32_t n_tasks, const uint64_t* records, uint32_t* fine_hist) {
  if (n_tasks == 0) return hipSuccess;
  if (kc.kx_pass && kc.key_words != 1) return hipErrorInvalidValue;
  const size_t sh = round_lds(kc.key_words) + ((size_t)1 << kc.fine_bits) * 4;
  const dim3 g(n_tasks), b(kExpandThreads);
  if (kc.key_words == 2)
    hipLaunchKernelGGL((k_fine_hist<2, 0>), g, b, sh, s, kc, tm, records, fine_hist);
  else if (kc.kx_pass == 1)
    hipLaunchKernelGGL((k_fine_hist<1, 1>), g, b, sh, s, kc, tm, records, fine_hist);
  else if (kc.kx_pass == 2)
    hipLaunchKernelGGL((k_fine_hist<1, 2>), g, b, sh, s, kc, tm, records, fine_hist);
  else
    hipLaunchKernelGGL((k_fine_hist<1, 0>), g, b, sh, s, kc, tm, records, fine_hist);
  return hipGetLastError();
}

hipError_t launch_plan_tiles(hipStream_t s, const KeyCfg& kc, const uint32_t* fine_hist,
                             const uint64_t* key_base, const uint64_t* tile_base,
                             uint16_t* tile_of_fine, Tile* tiles,
                             unsigned long long* tile_cursor) {
  const uint32_t nf = 1u << kc.fine_bits;
  const size_t sh = ((size_t)nf + 1) * 4 + ((size_t)nf + 2) * 2 * 2 + 16 * 4;
  hipLaunchKernelGGL(k_plan_tiles, dim3(kc.n_bins), dim3(256), sh, s, kc, fine_hist, key_base,
                     tile_base, tile_of_fine, tiles, tile_cursor);
  return hipGetLastError();
}

template <int KW, int MODE>
static void expand_launch(hipStream_t s, uint32_t grid, size_t sh, const KeyCfg& kc,
                          const TaskMap& tm, const uint64_t* records,
                          const uint16_t* tile_of_fine, const uint64_t* tile_base,
                          const uint64_t* key_base, uint32_t mt, uint32_t n_tasks,
                          unsigned long long* tile_cursor, uint64_t* keys, uint32_t* weights) {
  (void)hipFuncSetAttribute((const void*)k_expand_scatter<KW, MODE>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((k_expand_scatter<KW, MODE>), dim3(grid), dim3(kExpandThreads), sh, s, kc,
                     tm, records, tile_of_fine, tile_base, key_base, mt, n_tasks, tile_cursor,
                     keys, weights);
}

hipError_t launch_expand_scatter(hipStream_t s, const KeyCfg& kc, const TaskMap& tm,
                                 uint32_t n_tasks, const uint64_t* records,
                                 const uint16_t* tile_of_fine, const uint64_t* tile_base,
                                 const uint64_t* key_base, uint32_t max_tiles_per_bin,
                                 unsigned long long* tile_cursor, uint64_t* keys,
                                 uint32_t* weights) {
  if (n_tasks == 0) return hipSuccess;
  if (kc.kx_pass && kc.key_words != 1) return hipErrorInvalidValue;
  if (kc.kx_pass == 2 && !weights) return hipErrorInvalidValue;
  const uint32_t nf = 1u << kc.fine_bits;
  const uint32_t mt = max_tiles_per_bin < 1 ? 1 : max_tiles_per_bin;
  const size_t sh = expand_lds(kc.key_words, mt, nf);
  const uint32_t grid = kc.key_words == 2 ? (n_tasks + kXcds - 1) / kXcds * kXcds : n_tasks;
  if (kc.key_words == 2)
    expand_launch<2, 0>(s, grid, sh, kc, tm, records, tile_of_fine, tile_base, key_base, mt,
                        n_tasks, tile_cursor, keys, weights);
  else if (kc.kx_pass == 1)
    expand_launch<1, 1>(s, grid, sh, kc, tm, records, tile_of_fine, tile_base, key_base, mt,
                        n_tasks, tile_cursor, keys, weights);
  else if (kc.kx_pass == 2)
    expand_launch<1, 2>(s, grid, sh, kc, tm, records, tile_of_fine, tile_base, key_base, mt,
                        n_tasks, tile_cursor, keys, weights);
  else
    expand_launch<1, 0>(s, grid, sh, kc, tm, records, tile_of_fine, tile_base, key_base, mt,
                        n_tasks, tile_cursor, keys, weights);
  return hipGetLastError();
}

}  // namespace kmc
