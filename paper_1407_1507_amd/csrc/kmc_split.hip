// Distribution phase: signature scan of every read, super k-mer split,
// signature histogram of a sample, and scatter of super k-mer records into
// bins held in HBM.
//
// Method (KMC 2, Methods): the signature of a k-mer is the smallest
// canonical p-mer in it that is allowed (no AAA / ACA start, no AA except at
// the start); consecutive k-mers with the same signature form one super
// k-mer, which is sent to the bin of that signature (Fig. 1, "Sketch of the
// algorithm").  Signatures are merged into bins from a histogram of a small
// sample of the input.
//
// GPU mapping: one read per lane.  A lane walks its read once; per base it
// updates the rolling forward / reverse-complement p-mer, the canonical
// p-mer, and the running minimum over the current k-mer's p-mers (the
// minimum is re-scanned from the read only when its position leaves the
// window).  Records are staged per workgroup in LDS, grouped by bin, and
// written with one atomic reservation per (workgroup, bin).
#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

namespace {

// Byte access into the read set: whole aligned 32-bit words when seq is
// 4-byte aligned (never past the last byte's word), bytes otherwise.
struct SeqReader {
  const uint8_t* seq;
  uint64_t n;
  bool a4;
  uint64_t widx;
  uint32_t w;
  __device__ SeqReader(const uint8_t* s, uint64_t nb, bool al) : seq(s), n(nb), a4(al), widx(~0ull), w(0) {}
  __device__ __forceinline__ uint32_t get(uint64_t pos) {
    if (a4 && (pos | 3ull) < n) {
      uint64_t wi = pos >> 2;
      if (wi != widx) {
        widx = wi;
        w = reinterpret_cast<const uint32_t*>(seq)[wi];
      }
      return (w >> ((pos & 3u) << 3)) & 0xFFu;
    }
    return seq[pos];
  }
};

__device__ __forceinline__ uint32_t fetch_byte(const uint8_t* seq, uint64_t n, bool a4, uint64_t pos) {
  if (a4 && (pos | 3ull) < n) {
    uint32_t w = reinterpret_cast<const uint32_t*>(seq)[pos >> 2];
    return (w >> ((pos & 3u) << 3)) & 0xFFu;
  }
  return seq[pos];
}

// Scan bytes [x0, x1) of one read.  For every valid k-mer start j the sink
// sees kmer(j, signature); every super k-mer is passed to
// sink.superkmer(first k-mer start, number of k-mers, signature, forward key
// of the first k-mer, tail symbols after the first k-mer).  A super k-mer is
// also closed after w = k - p + 1 k-mers, so that it never holds more than
// 2k - p symbols (the count does not depend on where super k-mers are cut).
template <int KW, class Sink>
__device__ __forceinline__ void scan_read(const uint8_t* __restrict__ seq, uint64_t n_bases,
                                          uint64_t x0, uint64_t x1, const ScanCfg& C,
                                          Sink& sink) {
  typedef typename KeyOf<KW>::T K;
  const uint32_t k = C.k, p = C.p;
  const K kmask = key_mask<K>(k);
  const uint32_t rcs = 2 * p - 2;
  SeqReader rd(seq, n_bases, C.aligned4 != 0);
  uint32_t run = 0, fp = 0, rp = 0, minv = 0;
  uint64_t minpos = 0;
  uint32_t cur_n = 0, cur_sig = 0;
  uint64_t cur_start = 0;
  K F = 0, curF = 0, tail = 0;
  for (uint64_t x = x0; x < x1; ++x) {
    bool ok;
    const uint32_t c = decode_base(rd.get(x), ok);
    if (!ok) {
      if (cur_n) sink.superkmer(cur_start, cur_n, cur_sig, curF, tail);
      cur_n = 0;
      run = 0;
      continue;
    }
    ++run;
    fp = ((fp << 2) | c) & C.pmask;
    rp = (rp >> 2) | ((3u - c) << rcs);
    if (Sink::kNeedKeys) F = ((F << 2) | (K)c) & kmask;
    if (run >= p) {
      const uint32_t can = min(fp, rp);
      const uint32_t a = (!C.filter || sig_allowed(can, p)) ? can : C.sent;
      if (run == p || a <= minv) {  // ties keep the newest position
        minv = a;
        minpos = x + 1 - p;
      }
    }
    if (run < k) continue;
    const uint64_t j = x + 1 - k;
    if (minpos < j) {
      // the minimum left the window: re-scan the p-mers of k-mer j
      uint32_t f2 = 0, r2 = 0, m = 0xFFFFFFFFu;
      uint64_t mp = j;
      for (uint64_t y = j; y <= x; ++y) {
        bool ok2;
        const uint32_t c2 = decode_base(fetch_byte(seq, n_bases, C.aligned4 != 0, y), ok2);
        f2 = ((f2 << 2) | c2) & C.pmask;
        r2 = (r2 >> 2) | ((3u - c2) << rcs);
        if (y + 1 >= j + p) {
          const uint32_t can = min(f2, r2);
          const uint32_t a = (!C.filter || sig_allowed(can, p)) ? can : C.sent;
          if (a <= m) {
            m = a;
            mp = y + 1 - p;
          }
        }
      }
      minv = m;
      minpos = mp;
    }
    sink.kmer(j, minv);
    if (cur_n && minv == cur_sig && cur_n < C.w) {
      ++cur_n;
      if (Sink::kNeedKeys) tail = (tail << 2) | (K)c;
    } else {
      if (cur_n) sink.superkmer(cur_start, cur_n, cur_sig, curF, tail);
      cur_start = j;
      cur_n = 1;
      cur_sig = minv;
      curF = F;
      tail = 0;
    }
  }
  if (cur_n) sink.superkmer(cur_start, cur_n, cur_sig, curF, tail);
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

// ------------------------------------------------------------ sample hist

template <int KW>
struct HistSink {
  static constexpr bool kNeedKeys = false;
  uint32_t* hist;
  uint64_t kmers;
  __device__ void kmer(uint64_t, uint32_t) {}
  __device__ void superkmer(uint64_t, uint32_t n, uint32_t sig,
                            typename KeyOf<KW>::T, typename KeyOf<KW>::T) {
    atomicAdd(&hist[sig], n);
    kmers += n;
  }
};

template <int KW>
__global__ void __launch_bounds__(kScanThreads)
k_sig_hist(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
           uint64_t n_reads, uint64_t n_bases, uint64_t stride, ScanCfg C, uint32_t* hist,
           unsigned long long* sample_kmers) {
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * stride;
  HistSink<KW> sink{hist, 0};
  if (r < n_reads) scan_read<KW>(seq, n_bases, offsets[r], offsets[r + 1], C, sink);
  if (sink.kmers) atomicAdd(sample_kmers, (unsigned long long)sink.kmers);
}

// ------------------------------------------------------------ split count

template <int KW, bool LDS>
struct CountSink {
  static constexpr bool kNeedKeys = false;
  const uint32_t* map;
  uint32_t* lrec;
  uint32_t* lkmer;
  unsigned long long* grec;
  unsigned long long* gkmer;
  __device__ void kmer(uint64_t, uint32_t) {}
  __device__ void superkmer(uint64_t, uint32_t n, uint32_t sig,
                            typename KeyOf<KW>::T, typename KeyOf<KW>::T) {
    const uint32_t b = map[sig];
    if (LDS) {
      atomicAdd(&lrec[b], 1u);
      atomicAdd(&lkmer[b], n);
    } else {
      atomicAdd(&grec[b], 1ull);
      atomicAdd(&gkmer[b], (unsigned long long)n);
    }
  }
};

template <int KW, bool LDS>
__global__ void __launch_bounds__(kScanThreads)
k_split_count(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
              uint64_t n_reads, uint64_t n_bases, ScanCfg C, const uint32_t* __restrict__ map,
              unsigned long long* rec_cnt, unsigned long long* kmer_cnt) {
  extern __shared__ uint32_t lds[];
  uint32_t* lrec = lds;
  uint32_t* lkmer = lds + (LDS ? C.n_bins : 0);
  if (LDS) {
    for (uint32_t i = threadIdx.x; i < C.n_bins; i += blockDim.x) lrec[i] = lkmer[i] = 0;
    __syncthreads();
  }
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  CountSink<KW, LDS> sink{map, lrec, lkmer, rec_cnt, kmer_cnt};
  if (r < n_reads) scan_read<KW>(seq, n_bases, offsets[r], offsets[r + 1], C, sink);
  if (LDS) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < C.n_bins; i += blockDim.x) {
      if (lrec[i]) {
        atomicAdd(&rec_cnt[i], (unsigned long long)lrec[i]);
        atomicAdd(&kmer_cnt[i], (unsigned long long)lkmer[i]);
      }
    }
  }
}

// ---------------------------------------------------------- split scatter

template <int KW>
struct ScatterSink {
  static constexpr bool kNeedKeys = true;
  static constexpr int RW = 2 * KW;  // record words
  const uint32_t* map;
  uint32_t cap;
  uint32_t* lnum;     // staged records
  uint32_t* lcnt;     // per bin
  uint64_t* stage;    // cap * RW
  uint32_t* sbin;     // cap
  uint16_t* srank;    // cap
  unsigned long long* gcursor;
  uint64_t* records;
  __device__ void kmer(uint64_t, uint32_t) {}
  __device__ void superkmer(uint64_t, uint32_t n, uint32_t sig, typename KeyOf<KW>::T F,
                            typename KeyOf<KW>::T tail) {
    const uint32_t b = map[sig];
    const uint32_t idx = cap ? atomicAdd(lnum, 1u) : 0u;
    uint64_t rec[RW];
    make_record(rec, F, tail, n);
    if (idx < cap) {
      srank[idx] = (uint16_t)atomicAdd(&lcnt[b], 1u);
      sbin[idx] = b;
#pragma unroll
      for (int q = 0; q < RW; ++q) stage[(uint64_t)idx * RW + q] = rec[q];
    } else {
      // staging full: reserve this one record directly
      const uint64_t g = atomicAdd(&gcursor[b], 1ull);
#pragma unroll
      for (int q = 0; q < RW; ++q) records[g * RW + q] = rec[q];
    }
  }
};

template <int KW>
__global__ void __launch_bounds__(kScanThreads)
k_split_scatter(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
                uint64_t n_reads, uint64_t n_bases, ScanCfg C, const uint32_t* __restrict__ map,
                unsigned long long* gcursor, uint64_t* records, uint32_t cap) {
  constexpr int RW = 2 * KW;
  extern __shared__ uint64_t lds64[];
  // layout: stage[cap*RW] u64 | delta[n_bins] u64 | lcnt[n_bins] u32 | lbase[n_bins] u32 |
  //         sbin[cap] u32 | inv[cap] u16 | srank[cap] u16 | lnum, scan tmp
  uint64_t* stage = lds64;
  uint64_t* delta = stage + (uint64_t)cap * RW;
  uint32_t* lcnt = reinterpret_cast<uint32_t*>(delta + C.n_bins);
  uint32_t* lbase = lcnt + C.n_bins;
  uint32_t* sbin = lbase + C.n_bins;
  uint16_t* inv = reinterpret_cast<uint16_t*>(sbin + cap);
  uint16_t* srank = inv + cap;
  uint32_t* misc = reinterpret_cast<uint32_t*>(srank + cap);
  uint32_t* lnum = misc;
  uint32_t* tmp = misc + 1;

  for (uint32_t i = threadIdx.x; i < C.n_bins; i += blockDim.x) lcnt[i] = 0;
  if (threadIdx.x == 0) *lnum = 0;
  __syncthreads();

  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  ScatterSink<KW> sink{map, cap, lnum, lcnt, stage, sbin, srank, gcursor, records};
  if (r < n_reads) scan_read<KW>(seq, n_bases, offsets[r], offsets[r + 1], C, sink);
  __syncthreads();

  const uint32_t nst = min(*lnum, cap);
  for (uint32_t i = threadIdx.x; i < C.n_bins; i += blockDim.x) lbase[i] = lcnt[i];
  __syncthreads();
  block_exclusive_scan(lbase, C.n_bins, tmp);
  // one reservation per non-empty bin; delta maps a local slot to its global slot
  for (uint32_t i = threadIdx.x; i < C.n_bins; i += blockDim.x) {
    if (lcnt[i]) {
      const uint64_t g = atomicAdd(&gcursor[i], (unsigned long long)lcnt[i]);
      delta[i] = g - lbase[i];
    }
  }
  for (uint32_t i = threadIdx.x; i < nst; i += blockDim.x)
    inv[lbase[sbin[i]] + srank[i]] = (uint16_t)i;
  __syncthreads();
  // write records grouped by bin: consecutive lanes -> consecutive slots
  for (uint32_t q = threadIdx.x; q < nst; q += blockDim.x) {
    const uint32_t i = inv[q];
    const uint64_t g = delta[sbin[i]] + q;
#pragma unroll
    for (int w = 0; w < RW; ++w) records[g * RW + w] = stage[(uint64_t)i * RW + w];
  }
}

// Same output without LDS staging (for bin counts whose LDS counters do not
// fit): one atomic slot claim per record.
template <int KW>
__global__ void __launch_bounds__(kScanThreads)
k_split_scatter_direct(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
                       uint64_t n_reads, uint64_t n_bases, ScanCfg C,
                       const uint32_t* __restrict__ map, unsigned long long* gcursor,
                       uint64_t* records) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  ScatterSink<KW> sink{map, 0, nullptr, nullptr, nullptr, nullptr, nullptr, gcursor, records};
  if (r < n_reads) scan_read<KW>(seq, n_bases, offsets[r], offsets[r + 1], C, sink);
}

// ------------------------------------------------------------------ debug

template <int KW>
struct DebugSink {
  static constexpr bool kNeedKeys = false;
  uint32_t* sig;
  uint8_t* start;
  __device__ void kmer(uint64_t j, uint32_t s) { sig[j] = s; }
  __device__ void superkmer(uint64_t j0, uint32_t, uint32_t, typename KeyOf<KW>::T,
                            typename KeyOf<KW>::T) {
    if (start) start[j0] = 1;
  }
};

template <int KW>
__global__ void __launch_bounds__(kScanThreads)
k_debug_sigs(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
             uint64_t n_reads, uint64_t n_bases, ScanCfg C, uint32_t* sig, uint8_t* start) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  DebugSink<KW> sink{sig, start};
  if (r < n_reads) scan_read<KW>(seq, n_bases, offsets[r], offsets[r + 1], C, sink);
}

__global__ void k_check_offsets(const uint64_t* __restrict__ off, uint64_t n_reads,
                                uint64_t n_bases, uint32_t* err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_reads) return;
  bool bad = false;
  if (i == 0 && off[0] != 0) bad = true;
  if (i == n_reads && off[n_reads] != n_bases) bad = true;
  if (i < n_reads && off[i + 1] < off[i]) bad = true;
  if (bad) atomicOr(err, 1u);
}

uint32_t grid_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

}  // namespace

// --------------------------------------------------------------- launchers

hipError_t launch_sig_hist(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                           uint64_t n_reads, uint64_t n_bases, uint64_t stride,
                           const ScanCfg& cfg, uint32_t key_words, uint32_t* hist,
                           unsigned long long* sample_kmers) {
  const uint64_t n_sample = (n_reads + stride - 1) / stride;
  if (n_sample == 0) return hipSuccess;
  const uint32_t g = grid_for(n_sample, kScanThreads);
  if (key_words == 1)
    hipLaunchKernelGGL(k_sig_hist<1>, dim3(g), dim3(kScanThreads), 0, s, seq, offsets, n_reads,
                       n_bases, stride, cfg, hist, sample_kmers);
  else
    hipLaunchKernelGGL(k_sig_hist<2>, dim3(g), dim3(kScanThreads), 0, s, seq, offsets, n_reads,
                       n_bases, stride, cfg, hist, sample_kmers);
  return hipGetLastError();
}

hipError_t launch_split_count(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                              uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                              uint32_t key_words, const uint32_t* sig_to_bin,
                              unsigned long long* rec_cnt, unsigned long long* kmer_cnt) {
  if (n_reads == 0) return hipSuccess;
  const uint32_t g = grid_for(n_reads, kScanThreads);
  const bool lds = cfg.n_bins <= (uint32_t)kLdsBinsMax;
  const size_t sh = lds ? 2 * cfg.n_bins * sizeof(uint32_t) : 0;
  if (key_words == 1) {
    if (lds)
      hipLaunchKernelGGL((k_split_count<1, true>), dim3(g), dim3(kScanThreads), sh, s, seq,
                         offsets, n_reads, n_bases, cfg, sig_to_bin, rec_cnt, kmer_cnt);
    else
      hipLaunchKernelGGL((k_split_count<1, false>), dim3(g), dim3(kScanThreads), 0, s, seq,
                         offsets, n_reads, n_bases, cfg, sig_to_bin, rec_cnt, kmer_cnt);
  } else {
    if (lds)
      hipLaunchKernelGGL((k_split_count<2, true>), dim3(g), dim3(kScanThreads), sh, s, seq,
                         offsets, n_reads, n_bases, cfg, sig_to_bin, rec_cnt, kmer_cnt);
    else
      hipLaunchKernelGGL((k_split_count<2, false>), dim3(g), dim3(kScanThreads), 0, s, seq,
                         offsets, n_reads, n_bases, cfg, sig_to_bin, rec_cnt, kmer_cnt);
  }
  return hipGetLastError();
}

size_t split_scatter_lds(uint32_t key_words, uint32_t n_bins, uint32_t cap) {
  const uint32_t RW = 2 * key_words;
  return (size_t)cap * RW * 8 + (size_t)n_bins * 8 + (size_t)n_bins * 8 + (size_t)cap * 4 +
         (size_t)cap * 4 + 4 + 4 * (kScanThreads / 64) + 16;
}

hipError_t launch_split_scatter(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                                uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                                uint32_t key_words, const uint32_t* sig_to_bin,
                                unsigned long long* cursor, uint64_t* records) {
  if (n_reads == 0) return hipSuccess;
  const uint32_t g = grid_for(n_reads, kScanThreads);
  // staging shrinks when many bins need LDS counters (65535 bins x 16 B = 1 MB
  // does not fit: then the per-record path is taken for every record)
  uint32_t cap = key_words == 1 ? kStageCap1 : kStageCap2;
  while (cap > 256 && split_scatter_lds(key_words, cfg.n_bins, cap) > 64 * 1024) cap >>= 1;
  if (split_scatter_lds(key_words, cfg.n_bins, cap) > 64 * 1024) {
    if (key_words == 1)
      hipLaunchKernelGGL(k_split_scatter_direct<1>, dim3(g), dim3(kScanThreads), 0, s, seq,
                         offsets, n_reads, n_bases, cfg, sig_to_bin, cursor, records);
    else
      hipLaunchKernelGGL(k_split_scatter_direct<2>, dim3(g), dim3(kScanThreads), 0, s, seq,
                         offsets, n_reads, n_bases, cfg, sig_to_bin, cursor, records);
    return hipGetLastError();
  }
  const size_t sh = split_scatter_lds(key_words, cfg.n_bins, cap);
  if (key_words == 1)
    hipLaunchKernelGGL(k_split_scatter<1>, dim3(g), dim3(kScanThreads), sh, s, seq, offsets,
                       n_reads, n_bases, cfg, sig_to_bin, cursor, records, cap);
  else
    hipLaunchKernelGGL(k_split_scatter<2>, dim3(g), dim3(kScanThreads), sh, s, seq, offsets,
                       n_reads, n_bases, cfg, sig_to_bin, cursor, records, cap);
  return hipGetLastError();
}

hipError_t launch_debug_sigs(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                             uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                             uint32_t key_words, uint32_t* sig, uint8_t* start) {
  if (n_reads == 0) return hipSuccess;
  const uint32_t g = grid_for(n_reads, kScanThreads);
  if (key_words == 1)
    hipLaunchKernelGGL(k_debug_sigs<1>, dim3(g), dim3(kScanThreads), 0, s, seq, offsets,
                       n_reads, n_bases, cfg, sig, start);
  else
    hipLaunchKernelGGL(k_debug_sigs<2>, dim3(g), dim3(kScanThreads), 0, s, seq, offsets,
                       n_reads, n_bases, cfg, sig, start);
  return hipGetLastError();
}

hipError_t launch_check_offsets(hipStream_t s, const uint64_t* offsets, uint64_t n_reads,
                                uint64_t n_bases, uint32_t* err) {
  const uint32_t g = grid_for(n_reads + 1, 256);
  hipLaunchKernelGGL(k_check_offsets, dim3(g), dim3(256), 0, s, offsets, n_reads, n_bases, err);
  return hipGetLastError();
}

}  // namespace kmc
