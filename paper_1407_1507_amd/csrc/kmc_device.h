// Device-side helpers shared by the kernels of libkmc_hip.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kmc {

typedef unsigned __int128 u128;

template <int KW> struct KeyOf;
template <> struct KeyOf<1> { typedef uint64_t T; };
template <> struct KeyOf<2> { typedef u128 T; };

// A/C/G/T (either case) -> 0..3; ok = false for any other byte.
// (b >> 1) & 3 maps A,C,T,G to 0,1,2,3; x ^ (x >> 1) turns that into
// A,C,G,T = 0,1,2,3.  Valid letters after case folding: 'A','C','G','T' are
// 0x41 + {0, 2, 6, 19}.
__device__ __forceinline__ uint32_t decode_base(uint32_t b, bool& ok) {
  uint32_t u = (b & 0xDFu) - 0x41u;
  ok = (u < 20u) && ((0x80045u >> u) & 1u);
  uint32_t x = (b >> 1) & 3u;
  return x ^ (x >> 1);
}

// Is the canonical p-mer c (2p bits, leftmost symbol highest) allowed as a
// signature?  Excluded: a start of AAA or ACA, or AA at any offset other
// than 0 (Methods, "From minimizers to signatures").  AAA at the start is an
// AA at offset 1, so the pair test covers it.
__device__ __forceinline__ bool sig_allowed(uint32_t c, uint32_t p) {
  if (p < 3) return true;
  uint32_t a = ~(c | (c >> 1)) & 0x555555u & ((1u << (2 * p)) - 1u);  // symbol is A
  uint32_t aa = a & (a >> 2);          // bit 2i: symbols i and i+1 from the right are A
  if (aa & ((1u << (2 * (p - 2))) - 1u)) return false;  // pairs not touching the first symbol
  return (c >> (2 * (p - 3))) != 4u;   // first three symbols A C A
}

// Reverse complement of a 2k-bit key: complement every symbol, reverse the
// order of the 2-bit symbols, keep the low 2k bits.
__device__ __forceinline__ uint64_t revcomp64(uint64_t x, uint32_t k) {
  x = ~x;
  x = ((x >> 2) & 0x3333333333333333ull) | ((x & 0x3333333333333333ull) << 2);
  x = ((x >> 4) & 0x0F0F0F0F0F0F0F0Full) | ((x & 0x0F0F0F0F0F0F0F0Full) << 4);
  x = ((x >> 8) & 0x00FF00FF00FF00FFull) | ((x & 0x00FF00FF00FF00FFull) << 8);
  x = ((x >> 16) & 0x0000FFFF0000FFFFull) | ((x & 0x0000FFFF0000FFFFull) << 16);
  x = (x >> 32) | (x << 32);
  return x >> (64 - 2 * k);
}
__device__ __forceinline__ u128 revcomp128(u128 x, uint32_t k) {
  uint64_t hi = revcomp64((uint64_t)x, 32);          // reversed low word
  uint64_t lo = revcomp64((uint64_t)(x >> 64), 32);  // reversed high word
  u128 r = ((u128)hi << 64) | lo;
  return r >> (128 - 2 * k);
}
__device__ __forceinline__ uint64_t revcomp_key(uint64_t x, uint32_t k) { return revcomp64(x, k); }
__device__ __forceinline__ u128 revcomp_key(u128 x, uint32_t k) { return revcomp128(x, k); }

template <class K>
__device__ __forceinline__ K key_mask(uint32_t k) {
  return (2 * k >= 8 * sizeof(K)) ? ~K(0) : ((K(1) << (2 * k)) - 1);
}

// In-place exclusive scan of a[0..n) held in LDS by the whole block
// (blockDim.x threads, a multiple of 64).  tmp needs blockDim.x / 64 words.
// Returns the total to every thread.  Must be called by all threads.
__device__ inline uint32_t block_exclusive_scan(uint32_t* a, uint32_t n, uint32_t* tmp) {
  const uint32_t nt = blockDim.x, t = threadIdx.x;
  const uint32_t per = (n + nt - 1) / nt;
  const uint32_t b = t * per, e = min(n, b + per);
  uint32_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += a[i];
  // inclusive scan of the per-thread sums inside the wave
  const uint32_t lane = t & 63u, wid = t >> 6;
  uint32_t v = sum;
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += o;
  }
  if (lane == 63) tmp[wid] = v;
  __syncthreads();
  uint32_t wave_off = 0, total = 0;
  for (uint32_t w = 0; w < nt / 64; ++w) {
    uint32_t s = tmp[w];
    if (w < wid) wave_off += s;
    total += s;
  }
  uint32_t run = wave_off + v - sum;
  for (uint32_t i = b; i < e; ++i) {
    uint32_t x = a[i];
    a[i] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

}  // namespace kmc

namespace kmc {

// Exclusive scan of one value per thread over the block; returns the
// exclusive prefix and sets total.  tmp needs blockDim.x / 64 words.  Must be
// called by all threads.
__device__ inline uint32_t block_scan_one(uint32_t v, uint32_t* tmp, uint32_t& total) {
  const uint32_t t = threadIdx.x, lane = t & 63u, wid = t >> 6;
  uint32_t x = v;
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += o;
  }
  if (lane == 63) tmp[wid] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (uint32_t w = 0; w < blockDim.x / 64; ++w) {
    uint32_t s = tmp[w];
    if (w < wid) off += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}


// ------------------------------------------------ reads and records
// The 4 bytes of the aligned word at xw (xw % 4 == 0); bytes at or past
// n_bases read as 0 (an invalid symbol).  Whole-word loads need seq 4-byte
// aligned; otherwise bytes are loaded one by one.
__device__ __forceinline__ uint32_t load_word(const uint8_t* __restrict__ seq, uint64_t n,
                                              bool a4, uint64_t xw) {
  if (a4 && xw + 3 < n) return reinterpret_cast<const uint32_t*>(seq)[xw >> 2];
  uint32_t w = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (xw + q < n) w |= (uint32_t)seq[xw + q] << (8 * q);
  return w;
}

// The 16 bytes at x16 (x16 % 16 == 0), same conventions: one 16-byte load
// when seq is 16-byte aligned and the chunk lies inside it.
__device__ __forceinline__ uint4 load_chunk(const uint8_t* __restrict__ seq, uint64_t n,
                                            uint32_t align, uint64_t x16) {
  if (align >= 16 && x16 + 15 < n) return reinterpret_cast<const uint4*>(seq)[x16 >> 4];
  const bool a4 = align >= 4;
  return make_uint4(load_word(seq, n, a4, x16), load_word(seq, n, a4, x16 + 4),
                    load_word(seq, n, a4, x16 + 8), load_word(seq, n, a4, x16 + 12));
}

// Record of a super k-mer (2 words for k <= 32, 4 words for k > 32):
//   word group 0: forward key of the first k-mer (hi word first for 2 words);
//   word group 1: the n-1 symbols after the first k-mer, left aligned (first
//                 symbol in the top bits), with n in the low 8 bits.
// At most w - 1 = k - p tail symbols, so 2(k-p) + 8 bits fit one group.
__device__ __forceinline__ void make_record(uint64_t* r, uint64_t F, uint64_t tail, uint32_t n) {
  r[0] = F;
  r[1] = (n > 1 ? (tail << (64 - 2 * (n - 1))) : 0ull) | n;
}
__device__ __forceinline__ void make_record(uint64_t* r, u128 F, u128 tail, uint32_t n) {
  u128 t = (n > 1 ? (tail << (128 - 2 * (n - 1))) : (u128)0) | (u128)n;
  r[0] = (uint64_t)(F >> 64);
  r[1] = (uint64_t)F;
  r[2] = (uint64_t)(t >> 64);
  r[3] = (uint64_t)t;
}

// Two-bit codes of the 4 bytes of w (bytes known to be bases), the first
// byte's code in the top two of the 8 bits: the byte -> code map of
// decode_base on every byte at once, then one multiply gathers the four
// codes (byte i's code, at bit 8i, lands at bit 30 - 2i; no other partial
// product reaches bits 24..31).
__device__ __forceinline__ uint32_t pack4(uint32_t w) {
  const uint32_t x = (w >> 1) & 0x03030303u;
  const uint32_t c = x ^ ((x >> 1) & 0x01010101u);
  return (c * 0x40100401u) >> 24;
}

// The record of the super k-mer whose first k-mer starts at j0 and which
// holds n k-mers, rebuilt from the read: the L = k + n - 1 symbols from j0
// (all valid bases) are read in aligned 16-byte chunks and packed two bits
// each; the first k go to the forward key, the rest to the tail.
template <int KW>
__device__ void record_from_read(const uint8_t* __restrict__ seq, uint64_t n_bases,
                                 uint32_t align, uint64_t j0, uint32_t n, uint32_t k,
                                 uint64_t* rec) {
  typedef typename KeyOf<KW>::T K;
  const uint64_t j1 = j0 + k + n - 1;
  K F = 0, T = 0;
  uint32_t a = 0;  // symbols taken so far
  for (uint64_t x16 = j0 & ~15ull; x16 < j1; x16 += 16) {
    const uint4 ch = load_chunk(seq, n_bases, align, x16);
    // the chunk's 16 codes, first byte's in the top bits
    const uint32_t P = (pack4(ch.x) << 24) | (pack4(ch.y) << 16) | (pack4(ch.z) << 8) |
                       pack4(ch.w);
    const uint32_t sk = x16 < j0 ? (uint32_t)(j0 - x16) : 0u;      // bytes before j0
    const uint32_t e = x16 + 16 > j1 ? (uint32_t)(j1 - x16) : 16u;  // end byte (exclusive)
    const uint32_t c = e - sk;                                      // 1 .. 16 symbols
    const uint64_t v = ((uint64_t)P >> (2 * (16 - e))) & ((1ull << (2 * c)) - 1);
    const uint32_t toF = a < k ? min(c, k - a) : 0u, toT = c - toF;
    if (toF) F = (F << (2 * toF)) | (K)(v >> (2 * toT));
    if (toT) T = (T << (2 * toT)) | (K)(v & ((1ull << (2 * toT)) - 1));
    a += c;
  }
  make_record(rec, F, T, n);
}


}  // namespace kmc
