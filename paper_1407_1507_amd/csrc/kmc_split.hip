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
// updates the rolling forward / reverse-complement p-mer and the canonical
// p-mer, and takes the window minimum over the current k-mer's p-mers by van
// Herk / Gil-Werman blocks kept in a lane-private LDS slice (no window is
// re-scanned).  Finished super k-mers are queued per lane in LDS as (start,
// k-mer count, signature), grouped by bin at the end of the workgroup, and
// each record is rebuilt from the read as it is written, with one atomic
// reservation per (workgroup, bin).
#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

namespace {

// Scan bytes [x0, x1) of one read.  For every k-mer start j the sink sees
// kmer(j, signature) (0xFFFFFFFF if the k-mer holds an invalid byte; the sink
// ignores starts outside the read); every super k-mer is passed to
// sink.superkmer(first k-mer start, number of k-mers, signature, bin of the
// signature, forward key of the first k-mer, tail symbols after the first
// k-mer).  A super k-mer is also closed after w = k - p + 1 k-mers, so that it
// never holds more than 2k - p symbols (where super k-mers are cut does not
// change the counts).
//
// The lane walks aligned 16-byte chunks from the chunk holding x0, the load
// of the next chunk in flight while the current one is scanned; bytes outside
// [x0, x1) count as invalid, so no k-mer leaves the read and the loop body has
// no start/end special cases.
//
// Window minimum without data-dependent branches (van Herk / Gil-Werman):
// p-mer values are grouped in blocks of w; when a block completes its suffix
// minima are formed in place; the window of a k-mer spans the suffix of one
// block and the prefix of the next, so its minimum is min(suffix, running
// prefix minimum).  Each lane keeps one block in its own slice vh[0 .. w) of
// LDS: at offset j of a block it first reads the previous block's suffix
// minimum at j + 1 and then stores its own value at j, which the previous
// block no longer needs, so the suffix minima become the next block's
// prefix in place.  A p-mer holding an invalid byte is stored as 0
// and a valid one as (value + 1), so a window minimum of 0 flags an invalid
// k-mer and N bases need no separate branch.
template <int KW, class VT, class Sink>
__device__ __forceinline__ void scan_read(const uint8_t* __restrict__ seq, uint64_t n_bases,
                                          uint64_t x0, uint64_t x1, const ScanCfg& C, VT* vh,
                                          Sink& sink) {
  typedef typename KeyOf<KW>::T K;
  const uint32_t k = C.k, p = C.p, w = C.w;
  if (x1 < x0 + k) return;
  const K kmask = key_mask<K>(k);
  const uint32_t rcs = 2 * p - 2;
  for (uint32_t i = 0; i < w; ++i) vh[i] = (VT)0;
  uint32_t run = 0, fp = 0, rp = 0;
  uint32_t in_blk = 0, pre = 0;
  uint32_t cur_n = 0, cur_sig = 0, cur_bin = 0;
  uint64_t cur_start = 0;
  K F = 0, curF = 0, tail = 0;
  uint64_t xc = x0 & ~15ull;
  uint4 chunk = load_chunk(seq, n_bases, C.seq_align, xc);
  for (; xc < x1; xc += 16) {
    const uint4 next =
        xc + 16 < x1 ? load_chunk(seq, n_bases, C.seq_align, xc + 16) : make_uint4(0, 0, 0, 0);
    // bytes q of the chunk inside [x0, x1): bits lo .. hi - 1 (one 64-bit
    // comparison per chunk instead of two per byte)
    const uint32_t lo = x0 > xc ? (uint32_t)min(x0 - xc, (uint64_t)16) : 0u;
    const uint32_t hi = (uint32_t)min(x1 - xc, (uint64_t)16);
    const uint32_t inside = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
#pragma unroll
    for (uint32_t q = 0; q < 16; ++q) {
      const uint64_t x = xc + q;
      const uint32_t word = q < 4 ? chunk.x : q < 8 ? chunk.y : q < 12 ? chunk.z : chunk.w;
      bool ok;
      const uint32_t c = decode_base((word >> (8 * (q & 3))) & 0xFFu, ok);
      ok = ok && ((inside >> q) & 1u);
      run = ok ? run + 1 : 0;
      fp = ((fp << 2) | c) & C.pmask;
      rp = (rp >> 2) | ((3u - c) << rcs);
      if (Sink::kNeedKeys) F = ((F << 2) | (K)c) & kmask;
      const uint32_t can = min(fp, rp);
      const uint32_t v =
          run >= p ? ((!C.filter || sig_allowed(can, p)) ? can : C.sent) + 1u : 0u;
      pre = in_blk == 0 ? v : min(pre, v);
      uint32_t suf;
      if (in_blk == w - 1) {
        // the block is complete: its suffix minima in place; the window of
        // this k-mer is the whole block
        vh[in_blk] = (VT)v;
        uint32_t r = v;
        for (int i = (int)w - 2; i >= 0; --i) {
          r = min(r, (uint32_t)vh[i]);
          vh[i] = (VT)r;
        }
        suf = r;
      } else {
        suf = (uint32_t)vh[in_blk + 1];  // previous block's suffix minimum
        vh[in_blk] = (VT)v;
      }
      const uint32_t m = min(suf, pre);
      const uint64_t j = x + 1 - k;
      if (m == 0) {
        sink.kmer(j, 0xFFFFFFFFu, x0, x1);
        if (cur_n) sink.superkmer(cur_start, cur_n, cur_sig, cur_bin, curF, tail);
        cur_n = 0;
      } else {
        const uint32_t sig = m - 1;
        sink.kmer(j, sig, x0, x1);
        if (cur_n && sig == cur_sig && cur_n < w) {
          ++cur_n;
          if (Sink::kNeedKeys) tail = (tail << 2) | (K)c;
        } else {
          if (cur_n) sink.superkmer(cur_start, cur_n, cur_sig, cur_bin, curF, tail);
          cur_start = j;
          cur_n = 1;
          cur_sig = sig;
          cur_bin = sink.bin_of(sig);  // issued now, used when the super k-mer closes
          curF = F;
          tail = 0;
        }
      }
      if (++in_blk == w) {
        in_blk = 0;
      }
    }
    chunk = next;
  }
  if (cur_n) sink.superkmer(cur_start, cur_n, cur_sig, cur_bin, curF, tail);
}

// Lane-private LDS slices for the window buffer.  The slices of a wave's 64
// lanes are read and written at the same offset j together, so their stride
// decides the bank conflicts: an odd number of 32-bit words (32-bit values),
// or 2 mod 4 16-bit values (an odd number of words), puts the 64 lanes in 64
// different banks.  (A stride of w + 1 = 48 words at w = 47 put all 64 lanes
// in four banks.)
__host__ __device__ __forceinline__ uint32_t vh_stride(uint32_t w, uint32_t vt_bytes) {
  const uint32_t s = w + 1;
  return vt_bytes == 4 ? (s | 1u) : s + ((2u - s) & 3u);
}
template <class VT>
__device__ __forceinline__ VT* lane_vh(void* lds, uint32_t w) {
  return reinterpret_cast<VT*>(lds) + threadIdx.x * vh_stride(w, sizeof(VT));
}

// ------------------------------------------------------------ sample hist

// Signatures below kLdsSig (fewer when the window buffers leave less room
// for two workgroups per compute unit) are counted in the workgroup's LDS
// first: the smallest canonical m-mers are the most frequent minimizers, and
// their global counters would otherwise take most of the sample's atomics on
// a few addresses.
constexpr uint32_t kLdsSig = 4096;

template <int KW>
struct HistSink {
  static constexpr bool kNeedKeys = false;
  uint32_t* hist_k;   // k-mers per signature
  uint32_t* hist_r;   // super k-mers per signature
  uint32_t* lds_k;    // the same for signatures below kLdsSig, in LDS
  uint32_t* lds_r;
  uint32_t nl;        // signatures counted in LDS
  uint64_t kmers;
  __device__ void kmer(uint64_t, uint32_t, uint64_t, uint64_t) {}
  __device__ uint32_t bin_of(uint32_t) { return 0; }
  __device__ void superkmer(uint64_t, uint32_t n, uint32_t sig, uint32_t,
                            typename KeyOf<KW>::T, typename KeyOf<KW>::T) {
    if (sig < nl) {
      atomicAdd(&lds_k[sig], n);
      atomicAdd(&lds_r[sig], 1u);
    } else {
      atomicAdd(&hist_k[sig], n);
      atomicAdd(&hist_r[sig], 1u);
    }
    kmers += n;
  }
};

template <int KW, class VT>
__global__ void __launch_bounds__(256)
k_sig_hist(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
           uint64_t n_reads, uint64_t n_bases, uint64_t stride, ScanCfg C, uint32_t* hist,
           unsigned long long* sample, uint32_t nl) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds8[];
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * stride;
  const uint32_t n_sig = C.sent + 1;
  const size_t vb =
      ((size_t)blockDim.x * vh_stride(C.w, sizeof(VT)) * sizeof(VT) + 15) & ~(size_t)15;
  uint32_t* lk = reinterpret_cast<uint32_t*>(lds8 + vb);  // after the window buffers
  uint32_t* lr = lk + nl;
  for (uint32_t i = threadIdx.x; i < 2 * nl; i += blockDim.x) lk[i] = 0;
  __syncthreads();
  HistSink<KW> sink{hist, hist + n_sig, lk, lr, nl, 0};
  uint64_t bases = 0;
  if (r < n_reads) {
    bases = offsets[r + 1] - offsets[r];
    scan_read<KW, VT>(seq, n_bases, offsets[r], offsets[r + 1], C, lane_vh<VT>(lds8, C.w), sink);
  }
  if (sink.kmers) atomicAdd(&sample[0], (unsigned long long)sink.kmers);
  if (bases) atomicAdd(&sample[1], (unsigned long long)bases);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) {
    if (lr[i]) {
      atomicAdd(&hist[i], lk[i]);
      atomicAdd(&hist[n_sig + i], lr[i]);
    }
  }
}

// ---------------------------------------------------------- split scatter
// One pass: every super k-mer record goes to its bin's region, whose size was
// estimated from the sample.  cursor[b] counts every record of bin b; records
// past the region end are not written (the host then repeats the pass with
// the exact sizes the cursors report).

// A record that finds its lane's queue full goes straight to its bin: one
// global reservation.  Out of line: the scan loop calls it for a few reads
// only, and inlined into every unrolled base step it would bloat the loop.
template <int KW>
__device__ __noinline__ void spill_record(const uint8_t* __restrict__ seq, uint64_t n_bases,
                                          uint32_t align, uint32_t k, uint64_t j0, uint32_t n,
                                          uint32_t b, unsigned long long* gcursor,
                                          unsigned long long* gkmer, const uint64_t* cap_base,
                                          uint64_t* records) {
  constexpr int RW = 2 * KW;
  uint64_t rec[RW];
  record_from_read<KW>(seq, n_bases, align, j0, n, k, rec);
  atomicAdd(&gkmer[b], (unsigned long long)n);
  const uint64_t g = atomicAdd(&gcursor[b], 1ull);
  if (g < cap_base[b + 1]) {
#pragma unroll
    for (int w = 0; w < RW; ++w) records[g * RW + w] = rec[w];
  }
}

// Every super k-mer goes to its lane's own queue in LDS as (start in the
// read, k-mer count, signature): no atomics while the wave scans (emission
// is divergent, so it must be cheap) and no record words in LDS (the records
// are rebuilt from the read when they are written, which keeps the
// workgroup's LDS small enough for five workgroups per compute unit).  A
// full queue sends the record straight to its bin.
template <int KW, class VT>
struct SlotSink {
  static constexpr bool kNeedKeys = false;
  const uint32_t* map;
  uint32_t* sj;      // this lane's Q slots: start of the first k-mer in the read
  uint8_t* sn;       // k-mers of the super k-mer
  VT* ssig;          // signature (VT holds every signature)
  uint32_t q, Q;
  uint64_t x0;       // start of the lane's read
  const uint8_t* seq;
  uint64_t n_bases;
  uint32_t align, k;
  unsigned long long* gcursor;
  unsigned long long* gkmer;
  const uint64_t* cap_base;
  uint64_t* records;
  __device__ void kmer(uint64_t, uint32_t, uint64_t, uint64_t) {}
  __device__ uint32_t bin_of(uint32_t) { return 0; }
  __device__ void superkmer(uint64_t j0, uint32_t n, uint32_t sig, uint32_t,
                            typename KeyOf<KW>::T, typename KeyOf<KW>::T) {
    if (q < Q) {
      sj[q] = (uint32_t)(j0 - x0);
      sn[q] = (uint8_t)n;
      ssig[q] = (VT)sig;
      ++q;
      return;
    }
    spill_record<KW>(seq, n_bases, align, k, j0, n, map[sig], gcursor, gkmer, cap_base, records);
  }
};

// Records without a queue (bin counts whose LDS arrays do not fit).
template <int KW>
struct DirectSink {
  static constexpr bool kNeedKeys = true;
  static constexpr int RW = 2 * KW;
  const uint32_t* map;
  unsigned long long* gcursor;
  unsigned long long* gkmer;
  const uint64_t* cap_base;
  uint64_t* records;
  __device__ void kmer(uint64_t, uint32_t, uint64_t, uint64_t) {}
  __device__ uint32_t bin_of(uint32_t sig) { return map[sig]; }
  __device__ void superkmer(uint64_t, uint32_t n, uint32_t, uint32_t b, typename KeyOf<KW>::T F,
                            typename KeyOf<KW>::T tail) {
    uint64_t rec[RW];
    make_record(rec, F, tail, n);
    atomicAdd(&gkmer[b], (unsigned long long)n);
    const uint64_t g = atomicAdd(&gcursor[b], 1ull);
    if (g < cap_base[b + 1]) {
#pragma unroll
      for (int w = 0; w < RW; ++w) records[g * RW + w] = rec[w];
    }
  }
};

// Queue slots per lane: 2^3, or 2^4 for reads that give more super k-mers
// than 8 on average (a slot is 7 bytes of LDS: records are rebuilt from the
// read at write-out).
constexpr uint32_t kSplitQBitsMin = 3, kSplitQBitsMax = 4;
// A bin's slot offsets (region offset + a workgroup's slots) fit 31 bits.
static_assert(kMaxBinRecords + (256ull << kSplitQBitsMax) < (1ull << 31),
              "32-bit slot offsets of the lane scan");

// LDS of k_split_scatter: region U (the lanes' window buffers during the
// scan, then the per-bin arrays and the slot order) followed by the queues.
struct SplitLds {
  uint32_t u_bytes, sj_off, qn_off, tmp_off, ssig_off, sn_off, total;
};
__host__ __device__ inline SplitLds split_lds(uint32_t lanes, uint32_t Q, uint32_t n_bins,
                                              uint32_t vh_bytes, uint32_t vt_bytes) {
  SplitLds L;
  const uint32_t cap = lanes * Q;
  const uint32_t bins = n_bins * 4 + n_bins * 12 + cap * 4;  // delta | lcnt lbase lkm | inv srank
  L.u_bytes = ((vh_bytes > bins ? vh_bytes : bins) + 15) & ~15u;
  L.sj_off = L.u_bytes;
  L.qn_off = L.sj_off + cap * 4;
  L.tmp_off = L.qn_off + lanes * 4;
  L.ssig_off = L.tmp_off + 16;
  L.sn_off = L.ssig_off + ((cap * vt_bytes + 15) & ~15u);
  L.total = L.sn_off + ((cap + 15) & ~15u);
  return L;
}

template <int KW, class VT>
__global__ void __launch_bounds__(256)
k_split_scatter(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
                uint64_t n_reads, uint64_t n_bases, ScanCfg C, const uint32_t* __restrict__ map,
                unsigned long long* gcursor, unsigned long long* gkmer,
                const uint64_t* __restrict__ cap_base, uint64_t* records, uint32_t vh_bytes,
                uint32_t qb) {
  constexpr int RW = 2 * KW;
  const uint32_t Q = 1u << qb;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds8[];
  const uint32_t tid = threadIdx.x, nt = blockDim.x, cap = nt * Q;
  const SplitLds SL = split_lds(nt, Q, C.n_bins, vh_bytes, sizeof(VT));
  uint32_t* sj = reinterpret_cast<uint32_t*>(lds8 + SL.sj_off);
  uint32_t* qn = reinterpret_cast<uint32_t*>(lds8 + SL.qn_off);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(lds8 + SL.tmp_off);
  VT* ssig = reinterpret_cast<VT*>(lds8 + SL.ssig_off);  // signature, then bin
  uint8_t* sn = lds8 + SL.sn_off;

  const uint64_t r = (uint64_t)blockIdx.x * nt + tid;
  const uint64_t x0 = r < n_reads ? offsets[r] : 0;
  SlotSink<KW, VT> sink{map, sj + tid * Q, sn + tid * Q, ssig + tid * Q, 0, Q, x0, seq,
                        n_bases, C.seq_align, C.k, gcursor, gkmer, cap_base, records};
  if (r < n_reads)
    scan_read<KW, VT>(seq, n_bases, x0, offsets[r + 1], C, lane_vh<VT>(lds8, C.w), sink);
  qn[tid] = sink.q;
  __syncthreads();  // the window buffers are dead: region U becomes the bin arrays

  // delta[b]: global slot of local slot q is cap_base[b] + delta[b] + q, in
  // 32 bits.  The host keeps every region below kMaxBinRecords records, so a
  // reservation starting further into the bin than that lies wholly past the
  // region's end: its offset is clamped to kMaxBinRecords, which still lands
  // every slot past the end (not written; the cursor has counted them).
  int32_t* delta = reinterpret_cast<int32_t*>(lds8);
  uint32_t* lcnt = reinterpret_cast<uint32_t*>(delta + C.n_bins);
  uint32_t* lbase = lcnt + C.n_bins;
  uint32_t* lkm = lbase + C.n_bins;
  uint16_t* inv = reinterpret_cast<uint16_t*>(lkm + C.n_bins);
  uint16_t* srank = inv + cap;
  for (uint32_t i = tid; i < C.n_bins; i += nt) lcnt[i] = lkm[i] = 0;
  __syncthreads();
  // bins of the queued records, their rank inside the bin, k-mers per bin
  for (uint32_t i = tid; i < cap; i += nt) {
    if ((i & (Q - 1)) < qn[i >> qb]) {
      const uint32_t b = map[ssig[i]];
      ssig[i] = (VT)b;  // n_bins <= 65535
      srank[i] = (uint16_t)atomicAdd(&lcnt[b], 1u);
      atomicAdd(&lkm[b], (uint32_t)sn[i]);
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < C.n_bins; i += nt) lbase[i] = lcnt[i];
  __syncthreads();
  const uint32_t nst = block_exclusive_scan(lbase, C.n_bins, tmp);
  // one reservation per non-empty bin; delta maps a local slot to its global slot
  for (uint32_t i = tid; i < C.n_bins; i += nt) {
    if (lcnt[i]) {
      const uint64_t g = atomicAdd(&gcursor[i], (unsigned long long)lcnt[i]);
      const uint64_t rel = min(g - cap_base[i], (uint64_t)kMaxBinRecords);
      delta[i] = (int32_t)((int64_t)rel - (int64_t)lbase[i]);
    }
    if (lkm[i]) atomicAdd(&gkmer[i], (unsigned long long)lkm[i]);
  }
  for (uint32_t i = tid; i < cap; i += nt)
    if ((i & (Q - 1)) < qn[i >> qb]) inv[lbase[ssig[i]] + srank[i]] = (uint16_t)i;
  __syncthreads();
  // records grouped by bin: consecutive lanes -> consecutive slots; each is
  // rebuilt from its read
  const uint64_t r0 = (uint64_t)blockIdx.x * nt;
  for (uint32_t q = tid; q < nst; q += nt) {
    const uint32_t i = inv[q];
    const uint32_t b = ssig[i];
    const uint64_t g = (uint64_t)((int64_t)cap_base[b] + delta[b] + (int64_t)q);
    if (g < cap_base[b + 1]) {
      uint64_t rec[RW];
      record_from_read<KW>(seq, n_bases, C.seq_align, offsets[r0 + (i >> qb)] + sj[i], sn[i],
                           C.k, rec);
#pragma unroll
      for (int w = 0; w < RW; ++w) records[g * RW + w] = rec[w];
    }
  }
}

// Same output without LDS staging (bin counts whose LDS arrays do not fit).
template <int KW, class VT>
__global__ void __launch_bounds__(256)
k_split_scatter_direct(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
                       uint64_t n_reads, uint64_t n_bases, ScanCfg C,
                       const uint32_t* __restrict__ map, unsigned long long* gcursor,
                       unsigned long long* gkmer, const uint64_t* __restrict__ cap_base,
                       uint64_t* records) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds8[];
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  DirectSink<KW> sink{map, gcursor, gkmer, cap_base, records};
  if (r < n_reads)
    scan_read<KW, VT>(seq, n_bases, offsets[r], offsets[r + 1], C, lane_vh<VT>(lds8, C.w), sink);
}

// ------------------------------------------------------------------ debug

template <int KW>
struct DebugSink {
  static constexpr bool kNeedKeys = false;
  uint32_t* sig;
  uint8_t* start;
  __device__ void kmer(uint64_t j, uint32_t s, uint64_t x0, uint64_t x1) {
    if (j >= x0 && j < x1) sig[j] = s;  // starts before the read are not the read's
  }
  __device__ uint32_t bin_of(uint32_t) { return 0; }
  __device__ void superkmer(uint64_t j0, uint32_t, uint32_t, uint32_t, typename KeyOf<KW>::T,
                            typename KeyOf<KW>::T) {
    if (start) start[j0] = 1;
  }
};

template <int KW, class VT>
__global__ void __launch_bounds__(256)
k_debug_sigs(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets,
             uint64_t n_reads, uint64_t n_bases, ScanCfg C, uint32_t* sig, uint8_t* start) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds8[];
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  DebugSink<KW> sink{sig, start};
  if (r < n_reads)
    scan_read<KW, VT>(seq, n_bases, offsets[r], offsets[r + 1], C, lane_vh<VT>(lds8, C.w), sink);
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

// A lane walks a whole read one base per step, so long reads (a mean above
// kLongRead bases) take the position-per-lane scan, which walks a read 64
// bases per step.
constexpr uint64_t kLongRead = 2048;
// A lane walks its read one base per step, so the lane scan fills the chip
// only with many reads: a job of fewer reads (or a sample histogram of fewer
// sampled reads) takes the position-per-lane scan, whose wavefronts share
// the positions of a few reads (measured: 35K reads, 235 -> 93 us; 770K
// reads of 175 bp at k = 55 still favour the lane scan, 747 vs 917 us).
constexpr uint64_t kLaneScanMinReads = 1ull << 18;
constexpr uint64_t kLaneHistMinSample = 4096;

// Window buffers hold u16 when every stored value (4^p + 1 at most) fits.
static bool small_vt(const ScanCfg& c) { return c.sent + 1u <= 0xFFFFu; }
static size_t vh_bytes(const ScanCfg& c, uint32_t lanes) {
  const uint32_t vt = small_vt(c) ? 2 : 4;
  const size_t b = (size_t)lanes * vh_stride(c.w, vt) * vt;
  return (b + 15) & ~(size_t)15;
}

#define KMC_SCAN_DISPATCH(KERNEL, grid, lanes, sh, s, ...)                                    \
  do {                                                                                      \
    if (key_words == 1) {                                                                   \
      if (small_vt(cfg)) {                                                                  \
        (void)hipFuncSetAttribute((const void*)KERNEL<1, uint16_t>,                         \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sh));   \
        hipLaunchKernelGGL((KERNEL<1, uint16_t>), grid, lanes, sh, s, __VA_ARGS__);         \
      } else {                                                                              \
        (void)hipFuncSetAttribute((const void*)KERNEL<1, uint32_t>,                         \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sh));   \
        hipLaunchKernelGGL((KERNEL<1, uint32_t>), grid, lanes, sh, s, __VA_ARGS__);         \
      }                                                                                     \
    } else {                                                                                \
      if (small_vt(cfg)) {                                                                  \
        (void)hipFuncSetAttribute((const void*)KERNEL<2, uint16_t>,                         \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sh));   \
        hipLaunchKernelGGL((KERNEL<2, uint16_t>), grid, lanes, sh, s, __VA_ARGS__);         \
      } else {                                                                              \
        (void)hipFuncSetAttribute((const void*)KERNEL<2, uint32_t>,                         \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sh));   \
        hipLaunchKernelGGL((KERNEL<2, uint32_t>), grid, lanes, sh, s, __VA_ARGS__);         \
      }                                                                                     \
    }                                                                                       \
  } while (0)

// lanes per workgroup for the plain scan kernels: window buffers <= 64 KB
static uint32_t scan_lanes(const ScanCfg& c) {
  uint32_t lanes = 256;
  while (lanes > 64 && vh_bytes(c, lanes) > 64 * 1024) lanes >>= 1;
  return lanes;
}

hipError_t launch_sig_hist(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                           uint64_t n_reads, uint64_t n_bases, uint64_t stride,
                           const ScanCfg& cfg, uint32_t key_words, uint32_t* hist,
                           unsigned long long* sample) {
  const uint64_t n_sample = (n_reads + stride - 1) / stride;
  if (n_sample == 0) return hipSuccess;
  if (n_bases > kLongRead * n_reads || n_sample < kLaneHistMinSample)
    return launch_sig_hist_wide(s, seq, offsets, n_reads, stride, cfg, key_words, hist,
                                sample);
  const uint32_t lanes = scan_lanes(cfg);
  const size_t vb = vh_bytes(cfg, lanes);
  // LDS-counted signatures: up to kLdsSig, fewer if that keeps the
  // workgroup within 80 KB (two per compute unit)
  uint32_t nl = std::min<uint32_t>(cfg.sent + 1, kLdsSig);
  if (vb + (size_t)nl * 8 > 80 * 1024)
    nl = vb < 80 * 1024 - 8 * 256 ? (uint32_t)((80 * 1024 - vb) / 8) : 256u;
  const size_t sh = vb + (size_t)nl * 8;
  KMC_SCAN_DISPATCH(k_sig_hist, dim3(grid_for(n_sample, lanes)), dim3(lanes), sh, s, seq,
                    offsets, n_reads, n_bases, stride, cfg, hist, sample, nl);
  return hipGetLastError();
}

static size_t split_lds_bytes(const ScanCfg& c, uint32_t lanes, uint32_t qb) {
  return split_lds(lanes, 1u << qb, c.n_bins, (uint32_t)vh_bytes(c, lanes), small_vt(c) ? 2 : 4)
      .total;
}

// A super k-mer holds about w / 2 k-mers (Table 6: 6.7 per 100 bp read at
// k = 28, m = 7), so a read of mean length L gives about 2 (L - k + 1) / w + 1
// of them.  The lane scan queues 2^qb of them per lane in LDS and sends the
// rest one by one to global memory: the queue is the shortest that holds the
// expected count, and reads expected to overflow the longest queue (long
// reads for their k: 911K reads of 175 bp at k = 21, 4.2 ms against 1.1 ms
// with 8 slots) take the position-per-lane scan.  Returns 0 when none fits.
static uint32_t lane_queue_bits(const ScanCfg& c, uint64_t n_reads, uint64_t n_bases) {
  const uint64_t L = n_reads ? n_bases / n_reads : 0;
  for (uint32_t qb = kSplitQBitsMin; qb <= kSplitQBitsMax; ++qb)
    if (L < c.k || 2 * (L - c.k + 1) + c.w <= ((uint64_t)c.w << qb)) return qb;
  return 0;
}

// The lane-per-read scan is used when 256 lanes' window buffers (16-bit
// values for p <= 7, 32-bit above) and record queues fit at least two
// workgroups per compute unit; otherwise the scan with one position per lane
// (the same signatures and records).  Returns the queue bits, 0 for the
// position-per-lane scan.
static uint32_t lane_scan_bits(const ScanCfg& c, uint64_t n_reads, uint64_t n_bases) {
  if (n_bases > kLongRead * n_reads || n_reads < kLaneScanMinReads) return 0;
  const uint32_t qb = lane_queue_bits(c, n_reads, n_bases);
  return qb && split_lds_bytes(c, 256, qb) <= 80 * 1024 ? qb : 0;
}

hipError_t launch_split_scatter(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                                uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                                uint32_t key_words, const uint32_t* sig_to_bin,
                                unsigned long long* cursor, unsigned long long* kmer_cnt,
                                const uint64_t* cap_base, uint64_t* records) {
  if (n_reads == 0) return hipSuccess;
  const uint32_t qb = lane_scan_bits(cfg, n_reads, n_bases);
  if (qb == 0)
    return launch_split_wide(s, seq, offsets, n_reads, n_bases, cfg, key_words, sig_to_bin,
                             cursor, kmer_cnt, cap_base, records);
  // largest workgroup whose window buffers + queues fit 80 KB (at least two per CU)
  for (uint32_t lanes = 256; lanes >= 64; lanes >>= 1) {
    const size_t vb = vh_bytes(cfg, lanes);
    const size_t sh = split_lds_bytes(cfg, lanes, qb);
    if (sh <= 80 * 1024) {
      KMC_SCAN_DISPATCH(k_split_scatter, dim3(grid_for(n_reads, lanes)), dim3(lanes), sh, s,
                        seq, offsets, n_reads, n_bases, cfg, sig_to_bin, cursor, kmer_cnt,
                        cap_base, records, (uint32_t)vb, qb);
      return hipGetLastError();
    }
  }
  const uint32_t lanes = scan_lanes(cfg);
  const size_t sh = vh_bytes(cfg, lanes);
  KMC_SCAN_DISPATCH(k_split_scatter_direct, dim3(grid_for(n_reads, lanes)), dim3(lanes), sh, s,
                    seq, offsets, n_reads, n_bases, cfg, sig_to_bin, cursor, kmer_cnt, cap_base,
                    records);
  return hipGetLastError();
}

hipError_t launch_debug_sigs(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                             uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                             uint32_t key_words, uint32_t* sig, uint8_t* start) {
  if (n_reads == 0) return hipSuccess;
  if (lane_scan_bits(cfg, n_reads, n_bases) == 0)
    return launch_debug_wide(s, seq, offsets, n_reads, cfg, key_words, sig, start);
  const uint32_t lanes = scan_lanes(cfg);
  const size_t sh = vh_bytes(cfg, lanes);
  KMC_SCAN_DISPATCH(k_debug_sigs, dim3(grid_for(n_reads, lanes)), dim3(lanes), sh, s, seq,
                    offsets, n_reads, n_bases, cfg, sig, start);
  return hipGetLastError();
}

hipError_t launch_check_offsets(hipStream_t s, const uint64_t* offsets, uint64_t n_reads,
                                uint64_t n_bases, uint32_t* err) {
  const uint32_t g = grid_for(n_reads + 1, 256);
  hipLaunchKernelGGL(k_check_offsets, dim3(g), dim3(256), 0, s, offsets, n_reads, n_bases, err);
  return hipGetLastError();
}

}  // namespace kmc
