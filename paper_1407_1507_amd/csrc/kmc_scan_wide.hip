// Split for long windows: the signature scan with one position per lane.
//
// The lane-per-read scan (kmc_split.hip) keeps a block of w = k - p + 1
// window values per lane in LDS.  With p > 7 the values need 32 bits and with
// large k the window is long (w = 47 at k = 55, p = 9), so those buffers
// leave room for only a few wavefronts per compute unit.  This scan needs no
// per-lane state: one wavefront walks the bytes of a run of consecutive reads
// (one contiguous stretch of the input) 64 positions at a time, one position
// per lane, and everything a position needs from the positions before it
// comes from other lanes of the same or the previous 64-position chunk:
//   * the 2-bit codes of the 16 bases ending at x, by doubling (1, 2, 4, 8
//     positions back), give the forward p-mer; its reverse complement is a
//     bit reversal;
//   * the minimum over the w p-mers of the k-mer ending at x is a sparse-table
//     minimum: minima over 2, 4, ... 2^L positions by doubling, then the
//     minimum of two overlapping 2^L windows;
//   * lengths of valid runs (no invalid byte, no read start), run starts,
//     super k-mer starts and ends come from 64-bit ballots.
// Same signatures, same super k-mers (cut after w k-mers) and the same
// records as the lane-per-read scan (Methods: signatures, super k-mers;
// Fig. 1).
#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

namespace {

constexpr uint32_t kReadsPerWave = 16;
constexpr uint32_t kScanWaves = 4;  // wavefronts per workgroup
constexpr uint32_t kInvalidSig = 0xFFFFFFFFu;

// The value held by the lane of position x - d (1 <= d <= 63): this chunk for
// lanes >= d, the previous chunk (prev) otherwise.
__device__ __forceinline__ uint32_t back(uint32_t cur, uint32_t prev, uint32_t d, uint32_t lane) {
  const int src = (int)(((lane - d) & 63u) << 2);
  const uint32_t a = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)cur);
  const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)prev);
  return lane >= d ? a : b;
}

__device__ __forceinline__ int hb64(uint64_t m) { return 63 - __clzll((long long)m); }  // m != 0

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t i) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)i);
  return ((uint64_t)hi << 32) | lo;
}

// Reverse complement of a p-mer (2p bits, first symbol highest): complement,
// reverse the bit order, swap the two bits back inside every symbol.
__device__ __forceinline__ uint32_t rc_pmer(uint32_t f, uint32_t p) {
  uint32_t r = __builtin_bitreverse32(~f);
  r = ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
  return r >> (32 - 2 * p);
}

// The `len` codes ending at position z (z lowest), from the ring of packed
// 16-code words (ring[y & 255] holds the codes of y - 15 .. y).
__device__ __forceinline__ uint64_t ring_codes(const uint32_t* ring, int32_t z, uint32_t len,
                                               uint64_t*) {
  const uint64_t v = ((uint64_t)ring[(z - 16) & 255] << 32) | ring[z & 255];
  return len >= 32 ? v : v & ((1ull << (2 * len)) - 1);
}
__device__ __forceinline__ u128 ring_codes(const uint32_t* ring, int32_t z, uint32_t len, u128*) {
  const u128 lo = ((u128)ring[(z - 16) & 255] << 32) | ring[z & 255];
  const u128 hi = ((u128)ring[(z - 48) & 255] << 32) | ring[(z - 32) & 255];
  const u128 v = (hi << 64) | lo;
  return len >= 64 ? v : v & (((u128)1 << (2 * len)) - 1);
}

enum ScanMode { kSplitStaged = 0, kSplitDirect = 1, kHist = 2, kDebug = 3 };

struct ScanOut {
  // split
  const uint32_t* map;                 // signature -> bin
  unsigned long long* gcursor;         // next record slot of every bin
  unsigned long long* gkmer;           // k-mers of every bin
  const uint64_t* cap_base;            // region of bin b: [cap_base[b], cap_base[b+1])
  uint64_t* records;
  uint64_t n_bases;                    // bytes of seq (records are rebuilt from it)
  uint32_t cap;                        // staged records per workgroup
  // signature histogram of a sample: k-mers per signature, then super
  // k-mers per signature (n_sig each); sample[0] k-mers, sample[1] bases
  uint32_t* hist;
  uint32_t n_sig;
  unsigned long long* sample;
  // debug
  uint32_t* dsig;
  uint8_t* dstart;
};

// LDS of the staged split: the staged super k-mers as (first k-mer start,
// k-mer count, signature) (records are rebuilt from the reads when they are
// written, so no record words and no code rings are kept), per-bin counters
// and the record permutation.
struct StageLayout {
  uint64_t* start;      // cap: first k-mer start in seq
  uint64_t* delta;      // n_bins
  uint32_t* lcnt;       // n_bins
  uint32_t* lbase;      // n_bins
  uint32_t* lkm;        // n_bins
  uint32_t* ssig;       // cap: signature, then bin
  uint16_t* srank;      // cap
  uint16_t* inv;        // cap
  uint32_t* misc;       // [0] staged, [1] iterations, [2..] scan tmp
  uint8_t* sn;          // cap: k-mers
};

__device__ __forceinline__ StageLayout stage_layout(uint8_t* lds, uint32_t cap, uint32_t n_bins) {
  StageLayout L;
  L.start = reinterpret_cast<uint64_t*>(lds);
  L.delta = L.start + cap;
  L.lcnt = reinterpret_cast<uint32_t*>(L.delta + n_bins);
  L.lbase = L.lcnt + n_bins;
  L.lkm = L.lbase + n_bins;
  L.ssig = L.lkm + n_bins;
  L.srank = reinterpret_cast<uint16_t*>(L.ssig + cap);
  L.inv = L.srank + cap;
  L.misc = reinterpret_cast<uint32_t*>(L.inv + cap);
  L.sn = reinterpret_cast<uint8_t*>(L.misc + 2 + kScanWaves);
  return L;
}

// Write the staged records of the workgroup to their bins: one reservation
// per (flush, bin), consecutive lanes writing consecutive slots of a bin.
// All threads call it, with the staged records complete.
template <int KW>
__device__ void flush_stage(const StageLayout& L, const uint8_t* __restrict__ seq,
                            const ScanCfg& C, const ScanOut& O) {
  constexpr int RW = 2 * KW;
  const uint32_t tid = threadIdx.x, nt = blockDim.x, n_bins = C.n_bins;
  const uint32_t nst = L.misc[0];
  for (uint32_t i = tid; i < nst; i += nt) {
    const uint32_t b = O.map[L.ssig[i]];
    L.ssig[i] = b;
    L.srank[i] = (uint16_t)atomicAdd(&L.lcnt[b], 1u);
    atomicAdd(&L.lkm[b], (uint32_t)L.sn[i]);
  }
  __syncthreads();
  for (uint32_t b = tid; b < n_bins; b += nt) L.lbase[b] = L.lcnt[b];
  __syncthreads();
  block_exclusive_scan(L.lbase, n_bins, L.misc + 2);
  for (uint32_t b = tid; b < n_bins; b += nt) {
    if (L.lcnt[b]) {
      const uint64_t g = atomicAdd(&O.gcursor[b], (unsigned long long)L.lcnt[b]);
      L.delta[b] = g - L.lbase[b];
    }
    if (L.lkm[b]) atomicAdd(&O.gkmer[b], (unsigned long long)L.lkm[b]);
  }
  for (uint32_t i = tid; i < nst; i += nt) L.inv[L.lbase[L.ssig[i]] + L.srank[i]] = (uint16_t)i;
  __syncthreads();
  for (uint32_t q = tid; q < nst; q += nt) {
    const uint32_t i = L.inv[q];
    const uint32_t b = L.ssig[i];
    const uint64_t g = L.delta[b] + q;
    if (g < O.cap_base[b + 1]) {
      uint64_t rec[RW];
      record_from_read<KW>(seq, O.n_bases, C.seq_align, L.start[i], L.sn[i], C.k, rec);
#pragma unroll
      for (int w = 0; w < RW; ++w) O.records[g * RW + w] = rec[w];
    }
  }
  __syncthreads();
  for (uint32_t b = tid; b < n_bins; b += nt) L.lcnt[b] = L.lkm[b] = 0;
  if (tid == 0) L.misc[0] = 0;
  __syncthreads();
}

// The scan.  Wave g takes reads [g * rpw, (g+1) * rpw) (stride 1) or read
// g * stride alone.  Positions are k-mer ends: the k-mer ending at x covers
// bytes x - k + 1 .. x.  A super k-mer is emitted in the chunk that sees the
// position after its last k-mer.
template <int KW, int MODE>
__global__ void __launch_bounds__(kScanWaves * 64, 5)  // five workgroups per compute unit, as the LDS allows
k_scan(const uint8_t* __restrict__ seq, const uint64_t* __restrict__ offsets, uint64_t n_reads,
       ScanCfg C, uint32_t rpw, uint64_t stride, ScanOut O) {
  typedef typename KeyOf<KW>::T K;
  constexpr int RW = 2 * KW;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds8[];
  const uint32_t lane = __lane_id(), wid = threadIdx.x >> 6;
  const uint64_t gw = (uint64_t)blockIdx.x * kScanWaves + wid;
  uint64_t ra, rb;
  if (stride == 1) {
    ra = gw * rpw;
    rb = ra + rpw < n_reads ? ra + rpw : n_reads;
  } else {
    ra = gw * stride;
    rb = ra + 1;
  }
  if (ra >= n_reads) ra = rb = 0;
  const uint64_t x_begin = rb > ra ? offsets[ra] : 0;
  const uint64_t x_end = rb > ra ? offsets[rb] : 0;
  // read starts inside the stretch: lane i holds offsets[ra + 1 + i]
  const uint32_t nbnd = rb > ra + 1 ? (uint32_t)(rb - ra - 1) : 0;
  const uint64_t bnd = lane < nbnd ? offsets[ra + 1 + lane] : ~0ull;
  const uint32_t n_chunks = x_end > x_begin ? (uint32_t)((x_end - x_begin) >> 6) + 1 : 0;

  StageLayout L{};
  uint32_t* ring = nullptr;
  uint32_t iters = n_chunks;
  if (MODE == kSplitDirect) ring = reinterpret_cast<uint32_t*>(lds8) + wid * 256;
  if (MODE == kSplitStaged) {
    // the workgroup walks its chunks in step, so that staged records can be
    // flushed by all of its threads together
    L = stage_layout(lds8, O.cap, C.n_bins);
    for (uint32_t b = threadIdx.x; b < C.n_bins; b += blockDim.x) L.lcnt[b] = L.lkm[b] = 0;
    if (threadIdx.x == 0) L.misc[0] = L.misc[1] = 0;
    __syncthreads();
    if (lane == 0) atomicMax(&L.misc[1], n_chunks);
    __syncthreads();
    iters = L.misc[1];
  }

  const uint64_t le = ~0ull >> (63 - lane), lt = le >> 1;
  // positions relative to x_begin (a stretch is far shorter than 2^31 bytes)
  int32_t lastB = -1;  // last position no valid run reaches past
  int32_t lastRS = 0, lastST = 0;
  uint32_t pf1 = 0, pf2 = 0, pf4 = 0, pf8 = 0, psig = kInvalidSig, pL = 0;
  uint32_t pm[5] = {0, 0, 0, 0, 0};
  uint32_t bi = 0;
  uint64_t next_b = nbnd ? readlane64(bnd, 0) : ~0ull;
  const uint32_t dw = C.w - (1u << C.L);
  const uint32_t len = (uint32_t)(x_end - x_begin);
  // the byte of the next chunk is loaded one chunk ahead
  uint32_t bnext = lane < len ? seq[x_begin + lane] : 0u;
  uint32_t hk = 0;  // sampled k-mers of this lane (histogram mode)

  for (uint32_t it = 0; it < iters; ++it) {
    if (it < n_chunks) {
      const int32_t xc = (int32_t)(it << 6);
      const int32_t x = xc + (int32_t)lane;
      const uint32_t byte = bnext;
      if ((uint32_t)x + 64 < len) bnext = seq[x_begin + (uint32_t)x + 64];
      bool ok;
      const uint32_t c = decode_base(byte, ok);
      ok = ok && (uint32_t)x < len;
      uint64_t smask = 0;  // read starts in this chunk
      while (next_b < x_begin + (uint64_t)xc + 64) {
        smask |= 1ull << (next_b - x_begin - (uint64_t)xc);
        ++bi;
        next_b = bi < nbnd ? readlane64(bnd, bi) : ~0ull;
      }
      // valid run ending at x: no invalid byte and no read start inside it
      const uint64_t inv = ~__ballot(ok);
      if (smask & 1) lastB = xc - 1;
      const uint64_t mb = (inv & le) | ((smask >> 1) & lt);
      const int32_t B = mb ? xc + hb64(mb) : lastB;
      const uint32_t run = (uint32_t)(x - B);
      const uint64_t all = inv | (smask >> 1);
      if (all) lastB = xc + hb64(all);
      // codes of the 16 bases ending at x, forward and reverse-complement p-mer
      const uint32_t f2 = (back(c, pf1, 1, lane) << 2) | c;
      const uint32_t f4 = (back(f2, pf2, 2, lane) << 4) | f2;
      const uint32_t f8 = (back(f4, pf4, 4, lane) << 8) | f4;
      const uint32_t f16 = (back(f8, pf8, 8, lane) << 16) | f8;
      pf1 = c;
      pf2 = f2;
      pf4 = f4;
      pf8 = f8;
      if (MODE == kSplitDirect) ring[x & 255] = f16;
      const uint32_t fp = f16 & C.pmask;
      const uint32_t can = min(fp, rc_pmer(fp, C.p));
      const uint32_t v =
          run >= C.p ? ((!C.filter || sig_allowed(can, C.p)) ? can : C.sent) + 1u : 0u;
      // minimum over the w p-mers of the k-mer ending at x
      uint32_t m = v;
#pragma unroll
      for (uint32_t j = 0; j < 5; ++j) {
        if (j < C.L) {
          const uint32_t prev = pm[j];
          pm[j] = m;
          m = min(m, back(m, prev, 1u << j, lane));
        }
      }
      uint32_t wm = m;
      if (dw) wm = min(m, back(m, pL, dw, lane));
      pL = m;
      // signatures, run starts, super k-mer starts (a run is also cut every
      // w k-mers) and ends
      const bool kv = run >= C.k;
      const uint32_t sig = kv ? wm - 1u : kInvalidSig;
      const uint32_t sigp = back(sig, psig, 1, lane);
      psig = sig;
      const uint64_t RS = __ballot(kv && sigp != sig);
      const uint64_t rsle = RS & le;
      const int32_t lrs = rsle ? xc + hb64(rsle) : lastRS;
      if (RS) lastRS = xc + hb64(RS);
      bool st = false;
      if (kv) {
        const uint32_t d = (uint32_t)(x - lrs);
        st = d < C.w ? d == 0 : (d % C.w) == 0;
      }
      const uint64_t ST = __ballot(st);
      const bool e = sigp != kInvalidSig && (!kv || st);  // x - 1 ends a super k-mer
      const uint64_t E = __ballot(e);
      const uint64_t stlt = ST & lt;
      const int32_t s0 = stlt ? xc + hb64(stlt) : lastST;  // its first k-mer end
      if (ST) lastST = xc + hb64(ST);

      if (MODE == kDebug) {
        if (kv) O.dsig[x_begin + (uint32_t)(x - (int32_t)C.k + 1)] = sig;
        if (st) O.dstart[x_begin + (uint32_t)(x - (int32_t)C.k + 1)] = 1;
      }
      if (MODE == kHist && e) {
        const uint32_t n = (uint32_t)(x - s0);
        atomicAdd(&O.hist[sigp], n);
        atomicAdd(&O.hist[O.n_sig + sigp], 1u);
        hk += n;
      }
      if ((MODE == kSplitStaged || MODE == kSplitDirect) && E) {
        const int32_t y = x - 1;
        const uint32_t n = (uint32_t)(y - s0 + 1);
        if (MODE == kSplitStaged) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&L.misc[0], (uint32_t)__popcll(E));
          base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
          if (e) {
            const uint32_t idx = base + (uint32_t)__popcll(E & lt);
            L.start[idx] = x_begin + (uint64_t)(s0 - (int32_t)C.k + 1);
            L.sn[idx] = (uint8_t)n;
            L.ssig[idx] = sigp;
          }
        } else if (e) {
          __builtin_amdgcn_wave_barrier();  // the ring entries of this chunk are written
          uint64_t rec[RW];
          const K F = ring_codes(ring, s0, C.k, (K*)nullptr);
          const K T = n > 1 ? ring_codes(ring, y, n - 1, (K*)nullptr) : (K)0;
          make_record(rec, F, T, n);
          const uint32_t b = O.map[sigp];
          atomicAdd(&O.gkmer[b], (unsigned long long)n);
          const uint64_t g = atomicAdd(&O.gcursor[b], 1ull);
          if (g < O.cap_base[b + 1]) {
#pragma unroll
            for (int w = 0; w < RW; ++w) O.records[g * RW + w] = rec[w];
          }
        }
      }
    }
    if (MODE == kSplitStaged) {
      __syncthreads();
      if (L.misc[0] + kScanWaves * 64 > O.cap) flush_stage<KW>(L, seq, C, O);
    }
  }
  if (MODE == kSplitStaged) {
    __syncthreads();
    if (L.misc[0]) flush_stage<KW>(L, seq, C, O);
  }
  if (MODE == kHist) {
    uint32_t t = hk;
    for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
    if (lane == 0 && len) {
      atomicAdd(&O.sample[0], (unsigned long long)t);
      atomicAdd(&O.sample[1], (unsigned long long)len);
    }
  }
}

uint32_t wide_grid(uint64_t n, uint64_t per) { return (uint32_t)((n + per - 1) / per); }

template <int MODE>
hipError_t launch_scan(hipStream_t s, const uint8_t* seq, const uint64_t* offsets, uint64_t n_reads,
                       const ScanCfg& cfg, uint32_t key_words, uint64_t stride, size_t lds,
                       const ScanOut& o) {
  const uint64_t waves = stride == 1 ? (n_reads + kReadsPerWave - 1) / kReadsPerWave
                                     : (n_reads + stride - 1) / stride;
  if (waves == 0) return hipSuccess;
  const dim3 grid(wide_grid(waves, kScanWaves)), block(kScanWaves * 64);
  if (key_words == 1) {
    (void)hipFuncSetAttribute((const void*)k_scan<1, MODE>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_scan<1, MODE>), grid, block, lds, s, seq, offsets, n_reads, cfg,
                       kReadsPerWave, stride, o);
  } else {
    (void)hipFuncSetAttribute((const void*)k_scan<2, MODE>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_scan<2, MODE>), grid, block, lds, s, seq, offsets, n_reads, cfg,
                       kReadsPerWave, stride, o);
  }
  return hipGetLastError();
}

size_t stage_lds(uint32_t n_bins, uint32_t cap) {
  return (size_t)cap * 8 + (size_t)n_bins * 20 + (size_t)cap * 8 + (2 + kScanWaves) * 4 + cap + 16;
}

}  // namespace

// --------------------------------------------------------------- launchers

hipError_t launch_split_wide(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                             uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                             uint32_t key_words,
                             const uint32_t* sig_to_bin, unsigned long long* cursor,
                             unsigned long long* kmer_cnt, const uint64_t* cap_base,
                             uint64_t* records) {
  ScanOut o{};
  o.map = sig_to_bin;
  o.gcursor = cursor;
  o.gkmer = kmer_cnt;
  o.cap_base = cap_base;
  o.records = records;
  o.n_bases = n_bases;
  // the largest stage (records per flush) that keeps five workgroups per
  // compute unit, else four, else the largest within 64 KB; without room for
  // 512, records go straight to their bins
  for (size_t limit : {size_t(32) << 10, size_t(40) << 10, size_t(64) << 10}) {
    for (uint32_t cap = 2048; cap >= 512; cap >>= 1) {
      const size_t lds = stage_lds(cfg.n_bins, cap);
      if (lds <= limit) {
        o.cap = cap;
        return launch_scan<kSplitStaged>(s, seq, offsets, n_reads, cfg, key_words, 1, lds, o);
      }
    }
  }
  return launch_scan<kSplitDirect>(s, seq, offsets, n_reads, cfg, key_words, 1,
                                   (size_t)kScanWaves * 256 * 4, o);
}

hipError_t launch_sig_hist_wide(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                                uint64_t n_reads, uint64_t stride, const ScanCfg& cfg,
                                uint32_t key_words, uint32_t* hist, unsigned long long* sample) {
  ScanOut o{};
  o.hist = hist;
  o.n_sig = cfg.sent + 1;
  o.sample = sample;
  return launch_scan<kHist>(s, seq, offsets, n_reads, cfg, key_words, stride, 0, o);
}

hipError_t launch_debug_wide(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                             uint64_t n_reads, const ScanCfg& cfg, uint32_t key_words,
                             uint32_t* sig, uint8_t* start) {
  ScanOut o{};
  o.dsig = sig;
  o.dstart = start;
  return launch_scan<kDebug>(s, seq, offsets, n_reads, cfg, key_words, 1, 0, o);
}

}  // namespace kmc
