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

}  // namespace kmc
