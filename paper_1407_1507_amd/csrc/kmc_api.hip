// Host runtime of libkmc_hip.so: argument validation, the signature -> bin
// map, the per-job plan (bin, record, key and tile layout in HBM), the
// workspace cache and the C ABI declared in include/kmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/kmc.h"
#include "kmc_internal.h"

using namespace kmc;

// --------------------------------------------------------------- context

namespace {

enum BufId {
  B_SEQ, B_OFF, B_HIST, B_MAP, B_BINCNT, B_CURSOR, B_REC, B_FINE, B_TOF, B_TILES, B_TCUR,
  B_BASES, B_HTASK, B_ETASK, B_KEYS, B_COUNTS, B_TILEOUT, B_BIG, B_MISC, B_TMP, B_SCANTMP,
  B_TILEOFF, B_BINOFF, B_OUTK, B_OUTC, B_DBG1, B_DBG2, B_ASCSEG, B_ASCK, B_ASCC, B_STAGE,
  B_KXK, B_KXC, B_KXR, B_TMPW,
  B_AUX0, B_COUNT_ = B_AUX0 + kmc::kCtxAuxBuffers
};

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Misc device words (one small allocation): counters read back by the host.
struct Misc {
  unsigned long long sample_kmers;
  unsigned long long sample_bases;
  unsigned long long big_total;
  uint32_t n_big;
  uint32_t offsets_err;
  uint32_t big_next;  // work counter of the big-tile kernel
  uint32_t n_fail;    // big tiles left to the partition path (64-bit keys)
  unsigned long long big_out;  // entries kept by the big tiles
  uint32_t fail_next;  // work counter of the partition path
  uint32_t pad;
};

}  // namespace

// Carving of a caller-provided workspace: one region per buffer, sized by
// upper bounds computed from the job's sizes (kmc_workspace_size).
struct WsLayout {
  size_t off[B_COUNT_];
  size_t size[B_COUNT_];
  size_t total;
};

// Pinned host buffers for the small transfers between the phases (plans,
// counters, histograms), cached like the device buffers.
enum HostId { H_HIST, H_CNT, H_BASES, H_MISC, H_BINOFF, H_MAP, H_KX, H_COUNT_ };


struct kmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  DevBuf buf[B_COUNT_];
  DevBuf hbuf[H_COUNT_];  // pinned host memory
  hipEvent_t ev[32] = {};  // 0..5 phases, 8 + 2i / 9 + 2i kernel i, 28 / 29 gather
  // workspace mode (kmc_count_ws): buffers come from ws_base + layout
  uint8_t* ws_base = nullptr;
  WsLayout ws;
  // lent-region mode (an oversize served job): device buffers are taken from
  // the top of [pool_base, pool_base + pool_bytes); a bin group's buffers
  // start again at pool_mark, the top when the first group began
  uint8_t* pool_base = nullptr;
  size_t pool_bytes = 0, pool_top = 0, pool_mark = 0;
  bool ws_own_table = false;  // device table allocated apart from the workspace
  // allocation-free mode (kmc_count_static): host staging in pageable
  // vectors instead of pinned buffers, and the table written to the caller's
  // device buffers (user_cap entries)
  // memory budget (kmc_ctx_set_budget): device bytes a job's buffers may
  // take, 0 = unbounded; records beyond it spill to pinned host memory
  uint64_t budget = 0;
  // knobs of the counting path (never change the table): an override for
  // every job, else the tuned knobs of the job's class (kmc_autotune)
  bool has_knobs = false;
  kmc_knobs knobs{};
  std::map<uint32_t, kmc_knobs> tuned;
  uint32_t batch_workers = 0;  // 0 = the default pool size
  DevBuf spill;            // pinned host records (device-accessible)
  bool pageable_host = false;
  std::vector<uint8_t> hvec[H_COUNT_];
  uint64_t* user_keys = nullptr;
  uint32_t* user_counts = nullptr;
  uint64_t user_cap = 0;
  uint64_t user_need = 0;  // entries of a table that did not fit user_cap
  // extension slot (batch worker pool), released with the context
  void* ext = nullptr;
  void (*ext_free)(void*) = nullptr;
};

namespace {

struct Fail {
  kmc_status st;
};

void check(kmc_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    throw Fail{e == hipErrorOutOfMemory ? KMC_ERR_OUT_OF_MEMORY : KMC_ERR_DEVICE};
  }
}

template <class T>
T* ensure_host(kmc_ctx* c, HostId id, size_t bytes) {
  if (c->pageable_host) {
    std::vector<uint8_t>& v = c->hvec[id];
    if (v.size() < bytes) v.resize(bytes);
    return reinterpret_cast<T*>(v.data());
  }
  DevBuf& b = c->hbuf[id];
  if (b.cap < bytes) {
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    const size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
    check(c, hipHostMalloc(&b.p, want, 0), "hipHostMalloc");
    b.cap = want;
  }
  return static_cast<T*>(b.p);
}

template <class T>
T* ensure(kmc_ctx* c, BufId id, size_t bytes) {
  if (c->ws_base) {
    if (bytes > c->ws.size[id]) {
      c->err = "workspace too small for this job";
      throw Fail{KMC_ERR_OUT_OF_MEMORY};
    }
    return reinterpret_cast<T*>(c->ws_base + c->ws.off[id]);
  }
  DevBuf& b = c->buf[id];
  if (bytes == 0) bytes = 16;
  if (c->pool_base) {
    // exact sizes from the lent region; the top block grows in place, any
    // other block outgrown is left behind until its group ends
    if (b.p && b.cap >= bytes) return static_cast<T*>(b.p);
    const size_t want = (bytes + 255) & ~(size_t)255;
    if (b.p && static_cast<uint8_t*>(b.p) + b.cap == c->pool_base + c->pool_top &&
        static_cast<uint8_t*>(b.p) >= c->pool_base + c->pool_mark &&
        want - b.cap <= c->pool_bytes - c->pool_top) {
      c->pool_top += want - b.cap;
      b.cap = want;
      return static_cast<T*>(b.p);
    }
    if (want > c->pool_bytes - c->pool_top) {
      c->err = "the job's device buffers exceed the memory budget";
      throw Fail{KMC_ERR_OUT_OF_MEMORY};
    }
    b.p = c->pool_base + c->pool_top;
    b.cap = want;
    c->pool_top += want;
    return static_cast<T*>(b.p);
  }
  if (b.cap < bytes) {
    if (b.p) check(c, hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.cap = 0;
    size_t want = bytes + bytes / 8;
    want = (want + 4095) & ~(size_t)4095;
    check(c, hipMalloc(&b.p, want), "hipMalloc workspace");
    b.cap = want;
  }
  return static_cast<T*>(b.p);
}

// Lent-region mode: forget the buffers taken since pool_mark (those of the
// bin group that ended) and take the next group's from there.
void pool_next_group(kmc_ctx* c) {
  if (!c->pool_base) return;
  for (auto& b : c->buf)
    if (b.p && static_cast<uint8_t*>(b.p) >= c->pool_base + c->pool_mark) b = DevBuf{};
  c->pool_top = c->pool_mark;
}

// Device-accessible pinned host memory for records that do not fit the
// budget, cached like the device buffers.
template <class T = uint64_t>
T* ensure_spill(kmc_ctx* c, size_t bytes) {
  DevBuf& b = c->spill;
  if (b.cap < bytes) {
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    const size_t want = std::max<size_t>(bytes, 4096);
    check(c, hipHostMalloc(&b.p, want, hipHostMallocMapped), "hipHostMalloc records");
    b.cap = want;
  }
  void* d = nullptr;
  check(c, hipHostGetDevicePointer(&d, b.p, 0), "hipHostGetDevicePointer");
  return static_cast<T*>(d);
}

// Device bytes per k-mer of one bin group in the sorting phase: keys, their
// counters, the big-tile scratch, the group's gathered entries, and room for
// its records when they are staged from host memory.
uint64_t key_bytes_per_kmer(uint32_t kw) { return 3 * 8 * (uint64_t)kw + 8 + 16; }

uint32_t ilog2_ceil(uint64_t x) {
  uint32_t r = 0;
  while ((1ull << r) < x) ++r;
  return r;
}

// Signature -> bin map (Methods, "Sketch of the algorithm": the least
// frequent signatures of a sample are merged so that at most n_bins bins
// remain).  Reading: longest-processing-time packing of the sampled
// signatures, heaviest first (ties: smaller signature first), each into the
// currently lightest bin (ties: lowest bin id); signatures absent from the
// sample go to bin (signature mod n_bins).
void build_map(const uint32_t* hist, uint32_t n_sig, uint32_t n_bins, uint32_t* map) {
  std::vector<uint32_t> a, b;
  a.reserve(n_sig);
  uint32_t maxc = 0;
  for (uint32_t s = 0, m = 0; s < n_sig; ++s) {
    map[s] = m;  // s % n_bins, without a division per signature
    if (++m == n_bins) m = 0;
    if (hist[s]) {
      a.push_back(s);
      maxc = std::max(maxc, hist[s]);
    }
  }
  // seen signatures by descending count, ascending signature among equal
  // counts: a stable LSD radix sort on the complemented count
  b.resize(a.size());
  for (uint32_t shift = 0; shift < 32 && (maxc >> shift); shift += 11) {
    std::vector<uint32_t> cnt(2049, 0);
    for (uint32_t s : a) ++cnt[1 + ((~hist[s] >> shift) & 2047u)];
    for (uint32_t i = 0; i < 2048; ++i) cnt[i + 1] += cnt[i];
    for (uint32_t s : a) b[cnt[(~hist[s] >> shift) & 2047u]++] = s;
    a.swap(b);
  }
  // each to the lightest bin: the minimum of (load << 16 | bin) over the bins,
  // so equal loads go to the lowest bin id (n_bins <= 65535), kept by a
  // tournament tree (leaves = bins, each node the minimum of its children):
  // an update recomputes one path with branch-free minima, where a heap's
  // sift-down mispredicts a branch per level
  uint32_t nl = 1;
  while (nl < n_bins) nl <<= 1;
  std::vector<uint64_t> tree(2 * nl, ~0ull);
  for (uint32_t b = 0; b < n_bins; ++b) tree[nl + b] = b;
  for (uint32_t i = nl - 1; i >= 1; --i) tree[i] = std::min(tree[2 * i], tree[2 * i + 1]);
  for (uint32_t s : a) {
    const uint64_t top = tree[1];
    const uint32_t bin = (uint32_t)(top & 0xFFFFu);
    map[s] = bin;
    uint32_t i = nl + bin;
    tree[i] = top + ((uint64_t)hist[s] << 16);
    for (i >>= 1; i >= 1; i >>= 1) tree[i] = std::min(tree[2 * i], tree[2 * i + 1]);
  }
}

// Device tables are recycled: a freed table's memory (keys and counts in one
// block) goes to a per-process pool and serves a later table of a similar
// size, so that a stream of jobs does not pay a device allocation (and the
// synchronisation of a device free) per table.  The pool keeps at most
// kPoolKeep bytes per device; anything beyond that is freed at once.  Host
// tables come from the same pool's pinned host blocks (pseudo-device
// kHostPool): the table is copied straight into them at full bus rate, and a
// recycled block has no pages to fault in; tables above kPinnedMax bytes go
// to ordinary memory.
constexpr size_t kPoolKeep = size_t(8) << 30;
constexpr int kHostPool = 64;
constexpr size_t kPinnedMax = size_t(4) << 30;

struct TablePool {
  struct Block {
    int device;
    size_t bytes;
    void* p;
  };
  std::mutex mu;
  std::vector<Block> free_blocks;
  std::unordered_map<void*, Block> live;
  size_t kept[65] = {};  // per device, then the host blocks
};

TablePool& table_pool() {
  static TablePool* pool = new TablePool;  // never destroyed: tables may outlive everything
  return *pool;
}

void* pool_take(int device, size_t bytes) {
  TablePool& P = table_pool();
  {
    std::lock_guard<std::mutex> lk(P.mu);
    size_t best = SIZE_MAX;
    for (size_t i = 0; i < P.free_blocks.size(); ++i) {
      const auto& b = P.free_blocks[i];
      if (b.device == device && b.bytes >= bytes && b.bytes <= 2 * bytes + (1 << 20) &&
          (best == SIZE_MAX || b.bytes < P.free_blocks[best].bytes))
        best = i;
    }
    if (best != SIZE_MAX) {
      TablePool::Block b = P.free_blocks[best];
      P.free_blocks.erase(P.free_blocks.begin() + best);
      P.kept[device == kHostPool ? 64 : device & 63] -= b.bytes;
      P.live.emplace(b.p, b);
      return b.p;
    }
  }
  void* p = nullptr;
  const hipError_t e = device == kHostPool ? hipHostMalloc(&p, bytes, 0) : hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(P.mu);
  P.live.emplace(p, TablePool::Block{device, bytes, p});
  return p;
}

// Returns false if p did not come from the pool.
bool pool_give(void* p) {
  TablePool& P = table_pool();
  TablePool::Block b;
  std::vector<TablePool::Block> drop;
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return false;
    b = it->second;
    P.live.erase(it);
    P.free_blocks.push_back(b);
    const int ki = b.device == kHostPool ? 64 : b.device & 63;
    P.kept[ki] += b.bytes;
    // over the limit: free the oldest blocks of that device
    for (size_t i = 0; i < P.free_blocks.size() && P.kept[ki] > kPoolKeep;) {
      if (P.free_blocks[i].device == b.device) {
        P.kept[ki] -= P.free_blocks[i].bytes;
        drop.push_back(P.free_blocks[i]);
        P.free_blocks.erase(P.free_blocks.begin() + i);
      } else {
        ++i;
      }
    }
  }
  for (const auto& d : drop) {
    if (d.device == kHostPool) {
      (void)hipHostFree(d.p);
      continue;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(d.device);
    (void)hipFree(d.p);
    (void)hipSetDevice(cur);
  }
  return true;
}

// Host memory of a host table's keys and counts: one pinned block from the
// pool (reserved = 3) up to kPinnedMax bytes, else ordinary memory.
void host_table(kmc_table* T, uint64_t n, uint32_t kw) {
  const size_t kb = (std::max<uint64_t>(1, n * kw) * 8 + 255) & ~(size_t)255;
  const size_t total = kb + std::max<uint64_t>(1, n) * 4;
  void* blk = total <= kPinnedMax ? pool_take(kHostPool, total) : nullptr;
  if (blk) {
    T->keys = static_cast<uint64_t*>(blk);
    T->counts = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(blk) + kb);
    T->reserved = 3;
    return;
  }
  T->keys = static_cast<uint64_t*>(std::malloc(std::max<uint64_t>(1, n * kw) * 8));
  T->counts = static_cast<uint32_t*>(std::malloc(std::max<uint64_t>(1, n) * 4));
  T->reserved = 0;
  if (!T->keys || !T->counts) throw Fail{KMC_ERR_OUT_OF_MEMORY};
}

// The entries of a bin-grouped job in host memory: one pinned block of the
// table pool, keys then counts, that becomes the host table's block (a freed
// table's block serves the next grouped job, so its pages are pinned once).
struct HostEntries {
  // above this many bytes (or when pinning fails) keys and counts are two
  // ordinary allocations instead: pinning tens of GB would take host memory
  // from everything else
  static constexpr size_t kPinnedMax = size_t(16) << 30;
  void* blk = nullptr;  // pinned pool block, owned here until a table takes it
  bool pinned = false;
  uint64_t cap = 0;     // entries
  uint64_t* k = nullptr;
  uint32_t* c = nullptr;
  HostEntries() = default;
  HostEntries(const HostEntries&) = delete;
  HostEntries& operator=(const HostEntries&) = delete;
  ~HostEntries() { release(); }
  void release() {
    if (pinned) {
      if (blk) pool_give(blk);
    } else {
      std::free(k);
      std::free(c);
    }
    blk = nullptr;
    k = nullptr;
    c = nullptr;
    cap = 0;
  }
  // hand keys and counts to a host table (reserved 3: a pinned pool block,
  // 0: two allocations that kmc_table_free releases)
  void give_to(kmc_table* T) {
    T->keys = k;
    T->counts = c;
    T->reserved = pinned ? 3 : 0;
    blk = nullptr;
    k = nullptr;
    c = nullptr;
    cap = 0;
  }
  // room for n entries, the first keep of them kept; false if no memory
  bool reserve(uint64_t n, uint64_t keep, uint32_t kw) {
    if ((k || blk) && n <= cap) return true;
    const uint64_t ncap = std::max<uint64_t>(n, cap + cap / 2);
    const size_t kb = (std::max<uint64_t>(1, ncap * kw) * 8 + 255) & ~(size_t)255;
    const size_t total = kb + std::max<uint64_t>(1, ncap) * 4;
    void* nb = total <= kPinnedMax ? pool_take(kHostPool, total) : nullptr;
    uint64_t* nk;
    uint32_t* nc;
    if (nb) {
      nk = static_cast<uint64_t*>(nb);
      nc = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(nb) + kb);
    } else {
      nk = static_cast<uint64_t*>(std::malloc(kb));
      nc = static_cast<uint32_t*>(std::malloc(std::max<uint64_t>(1, ncap) * 4));
      if (!nk || !nc) {
        std::free(nk);
        std::free(nc);
        return false;
      }
    }
    if (keep) {
      std::memcpy(nk, k, keep * kw * 8);
      std::memcpy(nc, c, keep * 4);
    }
    release();
    blk = nb;
    pinned = nb != nullptr;
    cap = ncap;
    k = nk;
    c = nc;
    return true;
  }
};

kmc_table* new_table() {
  kmc_table* t = static_cast<kmc_table*>(std::calloc(1, sizeof(kmc_table)));
  return t;
}

struct Job {
  uint32_t k, p, n_bins, ci, cx, kw, flags, cmax;
  uint64_t n_reads, n_bases;
  const uint8_t* seq;     // device
  const uint64_t* off;    // device
  uint32_t seq_align;
};

ScanCfg scan_cfg(const Job& J) {
  ScanCfg C;
  C.k = J.k;
  C.p = J.p;
  C.w = J.k - J.p + 1;
  C.filter = (J.flags & KMC_FLAG_PLAIN_MINIMIZERS) ? 0u : 1u;
  C.pmask = (uint32_t)((1ull << (2 * J.p)) - 1);
  C.sent = 1u << (2 * J.p);
  C.n_bins = J.n_bins;
  C.seq_align = J.seq_align;
  C.L = 31u - (uint32_t)__builtin_clz(C.w);
  return C;
}

kmc_status validate(const kmc_reads* reads, const kmc_params* P) {
  if (!reads || !P) return KMC_ERR_INVALID_ARG;
  if (P->k < 4 || P->k > 64) return KMC_ERR_INVALID_ARG;
  if (P->p < 4 || P->p > 12 || P->p > P->k) return KMC_ERR_INVALID_ARG;
  const uint64_t n_sig = (1ull << (2 * P->p)) + 1;
  if (P->n_bins < 1 || P->n_bins > 65535 || P->n_bins > n_sig) return KMC_ERR_INVALID_ARG;
  if (P->cutoff_min > P->cutoff_max) return KMC_ERR_INVALID_ARG;
  if (P->flags & ~(KMC_FLAG_DEVICE_TABLE | KMC_FLAG_PLAIN_MINIMIZERS | KMC_FLAG_ASCENDING |
                   KMC_FLAG_NON_CANONICAL | KMC_FLAG_TEST_NARROW_FINGERPRINT | KMC_FLAG_KX_MASK))
    return KMC_ERR_INVALID_ARG;
  const uint32_t kx = (P->flags & KMC_FLAG_KX_MASK) >> 4;
  if (kx && ((P->flags & KMC_FLAG_NON_CANONICAL) || P->k + kx > 31)) return KMC_ERR_INVALID_ARG;
  if (reads->n_reads > 0 && (!reads->seq && reads->n_bases > 0)) return KMC_ERR_INVALID_ARG;
  if (reads->n_reads > 0 && !reads->offsets) return KMC_ERR_INVALID_ARG;
  if (reads->n_reads >= (1ull << 40) || reads->n_bases >= (1ull << 46)) return KMC_ERR_TOO_LARGE;
  if (!reads->on_device && reads->n_reads > 0) {
    const uint64_t* o = reads->offsets;
    if (o[0] != 0 || o[reads->n_reads] != reads->n_bases) return KMC_ERR_INVALID_ARG;
    for (uint64_t i = 0; i < reads->n_reads; ++i)
      if (o[i + 1] < o[i]) return KMC_ERR_INVALID_ARG;
  }
  return KMC_OK;
}

// Put the reads on the device (copy host reads into the workspace).
void stage_reads(kmc_ctx* c, const kmc_reads* R, Job& J) {
  J.n_reads = R->n_reads;
  J.n_bases = R->n_bases;
  if (R->on_device) {
    J.seq = R->seq;
    J.off = R->offsets;
  } else {
    uint8_t* s = ensure<uint8_t>(c, B_SEQ, R->n_bases + 16);
    uint64_t* o = ensure<uint64_t>(c, B_OFF, (R->n_reads + 1) * 8);
    if (R->n_bases)
      check(c, hipMemcpyAsync(s, R->seq, R->n_bases, hipMemcpyHostToDevice, c->stream), "H2D seq");
    if (R->offsets)
      check(c, hipMemcpyAsync(o, R->offsets, (R->n_reads + 1) * 8, hipMemcpyHostToDevice,
                              c->stream), "H2D offsets");
    else
      check(c, hipMemsetAsync(o, 0, 8, c->stream), "memset");
    J.seq = s;
    J.off = o;
  }
  J.seq_align = ((uintptr_t)J.seq & 15u) == 0 ? 16u : ((uintptr_t)J.seq & 3u) == 0 ? 4u : 1u;
}

void kbeg(kmc_ctx* c, int i, hipStream_t s) { check(c, hipEventRecord(c->ev[8 + 2 * i], s), "event"); }
void kend(kmc_ctx* c, int i, hipStream_t s) { check(c, hipEventRecord(c->ev[9 + 2 * i], s), "event"); }

float ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

// The class of a job for tuned knobs: key width and log2 of its bases.
uint32_t job_class(uint32_t kw, uint64_t n_bases) {
  uint32_t l = 0;
  while (l < 63 && (2ull << l) <= n_bases) ++l;
  return (kw - 1) * 64 + l;
}

// The knobs a job runs with (a workspace job always takes the defaults,
// which its workspace bounds assume).
kmc_knobs job_knobs(const kmc_ctx* c, uint32_t kw, uint64_t n_bases) {
  kmc_knobs k{0, 0, 0};
  if (c->ws_base) return k;
  if (c->has_knobs) return c->knobs;
  auto it = c->tuned.find(job_class(kw, n_bases));
  return it == c->tuned.end() ? k : it->second;
}

void run_count(kmc_ctx* c, const kmc_reads* R, const kmc_params* P, kmc_table* T) {
  Job J;
  J.k = P->k;
  J.p = P->p;
  J.n_bins = P->n_bins;
  J.ci = P->cutoff_min == 0 ? 1 : P->cutoff_min;
  J.cx = P->cutoff_max;
  J.cmax = P->counter_max == 0 ? 0xFFFFFFFFu : P->counter_max;
  J.kw = P->k <= 32 ? 1 : 2;
  J.flags = P->flags;
  hipStream_t s = c->stream;
  const uint32_t n_sig = (1u << (2 * J.p)) + 1;
  const uint32_t RW = 2 * J.kw;

  T->k = J.k;
  T->key_words = J.kw;
  T->n_bins = J.n_bins;
  T->p = J.p;
  T->on_device = (J.flags & KMC_FLAG_DEVICE_TABLE) ? 1 : 0;
  T->bin_offsets = static_cast<uint64_t*>(std::calloc(J.n_bins + 1, sizeof(uint64_t)));
  T->sig_to_bin = static_cast<uint32_t*>(std::calloc(n_sig, sizeof(uint32_t)));
  if (!T->bin_offsets || !T->sig_to_bin) throw Fail{KMC_ERR_OUT_OF_MEMORY};
  kmc_stats& st = T->stats;
  st.n_reads = R->n_reads;
  st.n_bases = R->n_bases;

  stage_reads(c, R, J);
  Misc* misc = ensure<Misc>(c, B_MISC, sizeof(Misc));
  check(c, hipMemsetAsync(misc, 0, sizeof(Misc), s), "memset");
  if (R->on_device && J.n_reads > 0)
    check(c, launch_check_offsets(s, J.off, J.n_reads, J.n_bases, &misc->offsets_err), "check");
  const ScanCfg C = scan_cfg(J);

  // ---- map: signature histograms of every s-th read (s = N/1e5 in [1,100])
  check(c, hipEventRecord(c->ev[0], s), "event");
  uint32_t* hist = ensure<uint32_t>(c, B_HIST, (size_t)n_sig * 8);
  check(c, hipMemsetAsync(hist, 0, (size_t)n_sig * 8, s), "memset");
  uint64_t stride = J.n_bases / 100000;
  stride = stride < 1 ? 1 : (stride > 100 ? 100 : stride);
  kbeg(c, KMC_K_SIG_HIST, s);
  check(c, launch_sig_hist(s, J.seq, J.off, J.n_reads, J.n_bases, stride, C, J.kw, hist,
                           &misc->sample_kmers), "sig_hist");
  kend(c, KMC_K_SIG_HIST, s);
  uint32_t* h_hist = ensure_host<uint32_t>(c, H_HIST, (size_t)n_sig * 8);
  Misc* h_misc_p = ensure_host<Misc>(c, H_MISC, sizeof(Misc));
  check(c, hipMemcpyAsync(h_hist, hist, (size_t)n_sig * 8, hipMemcpyDeviceToHost, s), "D2H");
  check(c, hipMemcpyAsync(h_misc_p, misc, sizeof(Misc), hipMemcpyDeviceToHost, s), "D2H");
  check(c, hipStreamSynchronize(s), "sync");
  Misc h_misc = *h_misc_p;
  if (h_misc.offsets_err) throw Fail{KMC_ERR_INVALID_ARG};
  st.sample_kmers = h_misc.sample_kmers;
  // the map is built in its pinned upload buffer, uploaded, then copied into
  // the table while the upload runs
  uint32_t* map = ensure_host<uint32_t>(c, H_MAP, (size_t)n_sig * 4);
  build_map(h_hist, n_sig, J.n_bins, map);
  uint32_t* d_map = ensure<uint32_t>(c, B_MAP, (size_t)n_sig * 4);
  check(c, hipMemcpyAsync(d_map, map, (size_t)n_sig * 4, hipMemcpyHostToDevice, s), "H2D map");
  check(c, hipEventRecord(c->ev[1], s), "event");
  std::memcpy(T->sig_to_bin, map, (size_t)n_sig * 4);

  // ---- split: one pass writing super k-mer records into bin regions sized
  // from the sample; if a bin overflows, the pass is repeated with the exact
  // sizes its cursor counted. A bin whose sample holds n records gets
  // scale * (1.15 n + 8 sqrt(n)) + 256: the relative error of a sampled count
  // shrinks as 1/sqrt(n), so small bins need the wider margin (reads of a
  // repeat family arrive together, which widens the spread beyond Poisson)
  std::vector<uint64_t> cap(J.n_bins, 0);
  {
    std::vector<double> est(J.n_bins, 0.0);
    const uint32_t* h_rec = h_hist + n_sig;  // sampled super k-mers per signature
    for (uint32_t g = 0; g < n_sig; ++g)
      if (h_rec[g]) est[map[g]] += h_rec[g];
    const double scale = h_misc.sample_bases ? (double)J.n_bases / (double)h_misc.sample_bases : 0.0;
    for (uint32_t b = 0; b < J.n_bins; ++b)
      cap[b] = std::min<uint64_t>((uint64_t)((1.15 * est[b] + 8.0 * std::sqrt(est[b])) * scale) + 256,
                                  kMaxBinRecords);
    if (c->ws_base) {
      // keep the regions inside the workspace; a bin that outgrows its share
      // takes the exact second pass, whose sizes always fit
      // (less one record per bin: the scaling below rounds each share)
      const uint64_t room = c->ws.size[B_REC] / (RW * 8) - J.n_bins;
      uint64_t total = 0;
      for (uint32_t b = 0; b < J.n_bins; ++b) total += cap[b];
      if (total > room)
        for (uint32_t b = 0; b < J.n_bins; ++b)
          cap[b] = (uint64_t)((double)cap[b] * (double)room / (double)total);
    }
  }
  // bases, n_bins + 1 entries each: record region base, key base, tile base,
  // record end, first fine-histogram task, first expansion task (pinned, so
  // the uploads are asynchronous; written only while the stream is idle)
  const size_t nb1 = (size_t)J.n_bins + 1, n_bases_words = 6 * nb1;
  uint64_t* rec_base = ensure_host<uint64_t>(c, H_BASES, n_bases_words * 8);
  unsigned long long* bincnt = ensure<unsigned long long>(c, B_BINCNT, (size_t)J.n_bins * 16);
  unsigned long long* cursor = bincnt;
  unsigned long long* kmer_dev = bincnt + J.n_bins;
  uint64_t* d_bases = ensure<uint64_t>(c, B_BASES, n_bases_words * 8);
  uint64_t* h_cnt = ensure_host<uint64_t>(c, H_CNT, (size_t)J.n_bins * 16);
  uint64_t* records = nullptr;
  bool rec_on_host = false;
  for (int pass = 0; pass < 2; ++pass) {
    rec_base[0] = 0;
    for (uint32_t b = 0; b < J.n_bins; ++b) rec_base[b + 1] = rec_base[b] + cap[b];
    // under a memory budget the records stay on the device while they take
    // at most half of it; beyond that they go to pinned host memory (the
    // split writes them over the bus, each bin group is staged back)
    const uint64_t rec_bytes = rec_base[J.n_bins] * RW * 8;
    rec_on_host = c->budget && !c->ws_base && rec_bytes > c->budget / 2;
    records = rec_on_host ? ensure_spill(c, rec_bytes) : ensure<uint64_t>(c, B_REC, rec_bytes);
    check(c, hipMemcpyAsync(d_bases, rec_base, ((size_t)J.n_bins + 1) * 8, hipMemcpyHostToDevice, s), "H2D");
    check(c, hipMemcpyAsync(cursor, rec_base, (size_t)J.n_bins * 8, hipMemcpyHostToDevice, s), "H2D");
    check(c, hipMemsetAsync(kmer_dev, 0, (size_t)J.n_bins * 8, s), "memset");
    kbeg(c, KMC_K_SPLIT, s);
    check(c, launch_split_scatter(s, J.seq, J.off, J.n_reads, J.n_bases, C, J.kw, d_map, cursor,
                                  kmer_dev, d_bases, records), "split_scatter");
    kend(c, KMC_K_SPLIT, s);
    check(c, hipMemcpyAsync(h_cnt, bincnt, (size_t)J.n_bins * 16, hipMemcpyDeviceToHost, s), "D2H");
    check(c, hipStreamSynchronize(s), "sync");
    bool over = false;
    for (uint32_t b = 0; b < J.n_bins; ++b) {
      const uint64_t used = h_cnt[b] - rec_base[b];
      if (used > cap[b]) over = true;
      cap[b] = used;
      if (used > kMaxBinRecords) {
        c->err = "a bin holds more super k-mers than a bin's region may address";
        throw Fail{KMC_ERR_TOO_LARGE};
      }
    }
    st.split_passes = pass + 1;
    if (!over) break;
  }
  std::vector<uint64_t> rec_cnt(cap);
  const uint64_t* kmer_cnt = h_cnt + J.n_bins;
  uint64_t max_bin = 0, n_rec = 0;
  std::vector<uint64_t> g_rec_base(rec_base, rec_base + nb1), g_key_base(nb1, 0);
  for (uint32_t b = 0; b < J.n_bins; ++b) {
    g_key_base[b + 1] = g_key_base[b] + kmer_cnt[b];
    max_bin = std::max<uint64_t>(max_bin, kmer_cnt[b]);
    n_rec += rec_cnt[b];
  }
  std::vector<uint64_t> g_kmers(kmer_cnt, kmer_cnt + J.n_bins);
  const uint64_t n_kmers = g_key_base[J.n_bins];
  st.n_kmers = n_kmers;
  st.n_superkmers = n_rec;
  st.max_bin_kmers = max_bin;
  if (max_bin >= (1ull << 32)) {
    c->err = "a bin holds 2^32 or more k-mers";
    throw Fail{KMC_ERR_TOO_LARGE};
  }
  check(c, hipEventRecord(c->ev[2], s), "event");

  KeyCfg kc;
  kc.k = J.k;
  kc.key_words = J.kw;
  kc.tile_cap = J.kw == 1 ? kTileCap1 : kTileCap2;
  const kmc_knobs kn = job_knobs(c, J.kw, J.n_bases);
  // the largest tile the tile kernels count is 3/4 of the table; knobs may
  // pack tiles to 2/4
  kc.tile_limit = (kn.tile_fill == 2 ? 2u : 3u) * kc.tile_cap / 4;
  kc.cutoff_min = J.ci;
  kc.cutoff_max = J.cx;
  kc.fp_bits = (J.flags & KMC_FLAG_TEST_NARROW_FINGERPRINT) ? 2u : 47u;
  kc.canonical = (J.flags & KMC_FLAG_NON_CANONICAL) ? 0u : 1u;
  kc.counter_max = J.cmax;
  // fine ranges of about tile_cap / 8 keys in the largest bin
  uint32_t fb = ilog2_ceil(max_bin * 8 / kc.tile_cap + 1);
  fb = (uint32_t)std::max<int32_t>(1, (int32_t)fb + std::max(-2, std::min(2, kn.fine_bits_bias)));
  fb = std::max<uint32_t>(1, std::min<uint32_t>({fb, (uint32_t)kMaxFineBits, 2 * J.k}));
  kc.fine_bits = fb;
  // big tiles of 64-bit keys take the streamed pass as a kernel of its own
  // when bins whose mean fine range exceeds half the tile limit hold an
  // eighth of the k-mers: most of their fine ranges are then big tiles, most
  // with few distinct keys.  Otherwise the big tiles are few (fine ranges
  // that hold the k-mers starting with the bin's signature), and one kernel
  // that streams or partitions each of them ends sooner.
  uint64_t heavy = 0;
  for (uint32_t b = 0; b < J.n_bins; ++b)
    if (g_kmers[b] > ((uint64_t)kc.tile_limit / 2 << fb)) heavy += g_kmers[b];
  const bool stream_big = heavy * 8 > n_kmers;
  // there, a big tile also takes the fine ranges after it up to four tile
  // limits of keys: a task's keys then land in fewer, longer runs per tile,
  // and fewer ranges just under the limit are left to the tile kernel; more
  // keys per big tile leave more of them above the table's distinct keys for
  // the streamed count (9-Gbase job: 219 -> 210 ms at four limits, 232 ms at
  // six)
  kc.big_merge = stream_big && J.kw == 1 ? 4 * kc.tile_limit : 0;

  // ---- groups of bins for the sorting phase.  Without a memory budget (or
  // when the job fits it) one group holds every bin.  Under a budget the bins
  // are taken in order into groups whose k-mers fit the key buffers the
  // budget leaves room for; each group is expanded, counted and assembled on
  // its own, its entries appended to the table (bins hold disjoint key sets,
  // so the table is the same).
  std::vector<std::pair<uint32_t, uint32_t>> groups;
  const uint64_t per_kmer = key_bytes_per_kmer(J.kw);
  uint64_t key_cap = ~0ull;
  if (c->budget && !c->ws_base) {
    // the records (unless spilled), host reads copied to the device, the
    // fine histograms, and a fixed allowance for the per-tile and per-task
    // arrays, scans and counters
    const uint64_t rec_dev = rec_on_host ? 0 : g_rec_base[J.n_bins] * RW * 8;
    // (per bin: up to three tiles beyond two per tile_limit keys, at under
    // 96 bytes of per-tile arrays each)
    const uint64_t fixed = (R->on_device ? 0 : J.n_bases + 8 * (J.n_reads + 1)) +
                           ((uint64_t)J.n_bins << fb) * 6 + (uint64_t)J.n_bins * 288 +
                           (16ull << 20);
    const uint64_t room = c->budget > rec_dev + fixed ? c->budget - rec_dev - fixed : 0;
    key_cap = room / per_kmer;
    if (max_bin > key_cap) {
      c->err = "a bin's k-mers do not fit the memory budget";
      throw Fail{KMC_ERR_TOO_LARGE};
    }
  }
  if (n_kmers <= key_cap) {
    groups.emplace_back(0u, J.n_bins);
  } else {
    uint32_t b0 = 0;
    uint64_t acc = 0;
    for (uint32_t b = 0; b < J.n_bins; ++b) {
      if (acc + g_kmers[b] > key_cap) {
        groups.emplace_back(b0, b);
        b0 = b;
        acc = 0;
      }
      acc += g_kmers[b];
    }
    groups.emplace_back(b0, J.n_bins);
  }
  const bool grouped = groups.size() > 1 || rec_on_host;
  const uint32_t kx = (J.flags & KMC_FLAG_KX_MASK) >> 4;
  if (kx && (grouped || c->ws_base)) {
    c->err = "(k,x)-mers need the job in one bin group and library-managed buffers";
    throw Fail{KMC_ERR_INVALID_ARG};
  }
  double kx_us[KMC_N_KERNELS] = {};
  st.n_groups = groups.size();
  st.records_spilled = rec_on_host ? 1 : 0;
  // a grouped job collects its entries in host memory, copied there straight
  // from the device, and builds the requested table from them at the end
  HostEntries acc;
  double acc_us[KMC_N_KERNELS] = {}, acc_phase[3] = {};
  uint64_t n_out_total = 0, n_distinct = 0, n_tiles_all = 0;
  uint64_t big_tiles = 0, big_keys = 0, big_out = 0;
  uint64_t* out_k = nullptr;
  uint32_t* out_c = nullptr;

  c->pool_mark = c->pool_top;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const uint32_t b0 = groups[gi].first, b1 = groups[gi].second, nbg = b1 - b0;
    const size_t gb1 = (size_t)nbg + 1;
    kc.n_bins = nbg;
    if (gi > 0) {
      check(c, hipMemsetAsync(misc, 0, sizeof(Misc), s), "memset");
      pool_next_group(c);  // the previous group's entries are in host memory
    }
    // the group's bases, relative to its first bin
    uint64_t* bases = ensure_host<uint64_t>(c, H_BASES, 6 * gb1 * 8);
    uint64_t* rb = bases;
    uint64_t* key_base = rb + gb1;
    uint64_t* tile_base = key_base + gb1;
    uint64_t* rec_end = tile_base + gb1;
    uint64_t* htask_pre = rec_end + gb1;
    uint64_t* etask_pre = htask_pre + gb1;
    uint64_t gmax = 0;
    for (uint32_t i = 0; i <= nbg; ++i) {
      rb[i] = g_rec_base[b0 + i] - g_rec_base[b0];
      key_base[i] = g_key_base[b0 + i] - g_key_base[b0];
    }
    uint64_t n_tiles = 0, max_tiles = 0;
    for (uint32_t i = 0; i < nbg; ++i) {
      const uint64_t km = g_kmers[b0 + i];
      gmax = std::max(gmax, km);
      tile_base[i] = n_tiles;
      // greedy packing: two consecutive tiles hold more than tile_limit keys;
      // and a tile holds at least one fine range, so a bin never has more
      // tiles than fine ranges (a bin whose fine ranges exceed the limit has
      // them as big tiles, sorted through HBM)
      uint64_t nt = km ? 2 * ((km - 1) / kc.tile_limit + 1) + 1 : 0;
      nt = std::min<uint64_t>(nt, 1ull << fb);
      n_tiles += nt;
      max_tiles = std::max(max_tiles, nt);
    }
    tile_base[nbg] = n_tiles;  // max_tiles <= 2^fb <= kMaxTilesPerBin
    n_tiles_all += n_tiles;
    const uint64_t gk = key_base[nbg];
    // the group's records: in place on the device, or staged from host memory
    const uint64_t* grec = records + g_rec_base[b0] * RW;
    if (rec_on_host) {
      const uint64_t words = rb[nbg] * RW;
      uint64_t* stage = ensure<uint64_t>(c, B_STAGE, std::max<uint64_t>(1, words) * 8);
      if (words)
        check(c, hipMemcpyAsync(stage, grec, words * 8, hipMemcpyDefault, s), "H2D records");
      grec = stage;
    }
    const std::vector<uint64_t> rs1(rb, rb + gb1);
    const std::vector<uint64_t> rc1(rec_cnt.begin() + b0, rec_cnt.begin() + b1);
    const uint64_t* d_key_base = d_bases + gb1;
    const uint64_t* d_tile_base = d_bases + 2 * gb1;
    // tasks: fine-histogram tasks of up to hrec records, expansion tasks of
    // one record per lane; only per-bin task offsets go to the device, which
    // lists every task's bin itself
    const uint64_t hrec = std::min<uint64_t>(65536, std::max<uint64_t>(1024, 8ull << fb));
    // expansion tasks: with heavy bins (thousands of tiles each, see above)
    // a task of 256 records lands less than one key per tile, and 512-record
    // tasks (two rounds) measured faster there (9-Gbase job 74.2 -> 62.7 ms)
    const uint64_t eper = kn.expand_task             ? kn.expand_task
                          : (stream_big && J.kw == 1) ? 2 * (uint64_t)kExpandThreads
                                                      : expand_task_records(J.kw);
    Tile* tiles = nullptr;
    uint64_t* tile_off = nullptr;
    uint64_t* keys = nullptr;
    uint32_t* counts = nullptr;
    uint64_t* h_binoff = nullptr;
    // One pass of the sorting phase over a record source (records of RW
    // words): bin i holds rcnt[i] records from record rstart[i] on.  Fine
    // histogram, tiles, expansion, counting, tile and bin offsets; reads
    // back the bin offsets of the counted entries (the distinct count in
    // h_binoff[gb1]) and the counters.  Keys are placed by the bins' k-mer
    // counts, which bound the keys of every pass.
    auto tile_pass = [&](const uint64_t* src, const uint64_t* rstart, const uint64_t* rcnt,
                         const KeyCfg& kp, bool weighted) {
    htask_pre[0] = etask_pre[0] = 0;
    for (uint32_t i = 0; i < nbg; ++i) {
      const uint64_t rc = rcnt[i];
      rb[i] = rstart[i];
      rec_end[i] = rb[i] + rc;
      htask_pre[i + 1] = htask_pre[i] + (rc + hrec - 1) / hrec;
      etask_pre[i + 1] = etask_pre[i] + (rc + eper - 1) / eper;
    }
    rb[nbg] = rec_end[nbg] = rstart[nbg];
    const uint64_t n_htasks = htask_pre[nbg], n_etasks = etask_pre[nbg];
    check(c, hipMemcpyAsync(d_bases, bases, 6 * gb1 * 8, hipMemcpyHostToDevice, s), "H2D");
    uint16_t* d_hbin = ensure<uint16_t>(c, B_HTASK, std::max<uint64_t>(1, n_htasks) * 2);
    ExpandTask* d_etask =
        ensure<ExpandTask>(c, B_ETASK, std::max<uint64_t>(1, n_etasks) * sizeof(ExpandTask));
    check(c, launch_task_bins(s, nbg, d_bases + 4 * gb1, d_hbin, d_bases + 5 * gb1, d_bases,
                              d_bases + 3 * gb1, (uint32_t)eper, d_etask),
          "task_bins");
    const TaskMap hmap{d_hbin, d_bases + 4 * gb1, d_bases, d_bases + 3 * gb1, (uint32_t)hrec,
                       nullptr};
    const TaskMap emap{nullptr, d_bases + 5 * gb1, d_bases, d_bases + 3 * gb1,
                       (uint32_t)eper, d_etask};
    const size_t nfine = (size_t)nbg << fb;
    uint32_t* fine = ensure<uint32_t>(c, B_FINE, nfine * 4);
    check(c, hipMemsetAsync(fine, 0, nfine * 4, s), "memset");
    kbeg(c, KMC_K_FINE_HIST, s);
    check(c, launch_fine_hist(s, kp, hmap, (uint32_t)n_htasks, src, fine), "fine_hist");
    kend(c, KMC_K_FINE_HIST, s);
    uint16_t* tof = ensure<uint16_t>(c, B_TOF, nfine * 2);
    tiles = ensure<Tile>(c, B_TILES, n_tiles * sizeof(Tile));
    unsigned long long* tcur = ensure<unsigned long long>(c, B_TCUR, n_tiles * 8);
    if (n_tiles) check(c, hipMemsetAsync(tiles, 0, n_tiles * sizeof(Tile), s), "memset");
    kbeg(c, KMC_K_PLAN_TILES, s);
    check(c, launch_plan_tiles(s, kp, fine, d_key_base, d_tile_base, tof, tiles, tcur), "plan");
    kend(c, KMC_K_PLAN_TILES, s);
    keys = ensure<uint64_t>(c, B_KEYS, gk * J.kw * 8);
    counts = ensure<uint32_t>(c, B_COUNTS, gk * 4);
    kbeg(c, KMC_K_EXPAND, s);
    check(c, launch_expand_scatter(s, kp, emap, (uint32_t)n_etasks, src, tof, d_tile_base,
                                   d_key_base, (uint32_t)max_tiles, tcur, keys,
                                   weighted ? counts : nullptr), "expand");
    kend(c, KMC_K_EXPAND, s);
    check(c, hipEventRecord(c->ev[3], s), "event");

    // ---- sort: tiles in LDS, big tiles through HBM
    uint32_t* tile_out = ensure<uint32_t>(c, B_TILEOUT, n_tiles * 8 + 8);
    uint32_t* tile_dist = tile_out + n_tiles + (n_tiles & 1);
    uint32_t* big = ensure<uint32_t>(c, B_BIG, n_tiles * 20 + 16);
    uint64_t* big_off = reinterpret_cast<uint64_t*>(big + ((n_tiles + 1) & ~1ull));
    uint32_t* big_order = reinterpret_cast<uint32_t*>(big_off + n_tiles);
    // the big tiles' sizes, read once to order them; the same words then hold
    // the list of big tiles left to the partition kernel
    uint32_t* big_size = big_order + n_tiles;
    uint32_t* big_fail = big_size;
    kbeg(c, KMC_K_TILE_SORT, s);
    check(c, launch_tile_sort(s, kp, tiles, n_tiles, keys, counts, tile_out, big, big_off,
                              &misc->n_big, &misc->big_total, tile_dist, big_size, weighted),
          "tile_sort");
    kend(c, KMC_K_TILE_SORT, s);
    // big tiles: their number stays on the device (no round trip); scratch
    // for their partition passes is sized for every key of the group
    kbeg(c, KMC_K_BIG_TILES, s);
    {
      uint64_t* tmp = ensure<uint64_t>(c, B_TMP, std::max<uint64_t>(1, gk) * J.kw * 8);
      uint32_t* tmpw =
          weighted ? ensure<uint32_t>(c, B_TMPW, std::max<uint64_t>(1, gk) * 4) : nullptr;
      check(c, launch_big_tiles(s, kp, tiles, big, big_off, big_size, big_order, big_fail,
                                &misc->n_big,
                                &misc->big_next, &misc->n_fail, &misc->fail_next, n_tiles,
                                stream_big, keys, tmp, counts, tmpw, tile_out, tile_dist,
                                &misc->big_out),
            "big_tiles");
    }
    kend(c, KMC_K_BIG_TILES, s);
    check(c, hipEventRecord(c->ev[4], s), "event");

    // ---- assemble: offsets of every tile's output, bin offsets, gather
    tile_off = ensure<uint64_t>(c, B_TILEOFF, (n_tiles + 1) * 8);
    uint64_t* scan_tmp = ensure<uint64_t>(c, B_SCANTMP, scan_tmp_words(n_tiles) * 8);
    kbeg(c, KMC_K_ASSEMBLE, s);
    check(c, launch_scan_u32(s, tile_out, n_tiles, tile_off, scan_tmp), "scan");
    uint64_t* bin_off = ensure<uint64_t>(c, B_BINOFF, gb1 * 8);
    check(c, launch_bin_offsets(s, tile_off, d_tile_base, nbg, bin_off), "bin_offsets");
    kend(c, KMC_K_ASSEMBLE, s);
    h_binoff = ensure_host<uint64_t>(c, H_BINOFF, (gb1 + 1) * 8);
    check(c, hipMemcpyAsync(h_binoff, bin_off, gb1 * 8, hipMemcpyDeviceToHost, s), "D2H");
    // distinct keys: sum of the per-tile counts (a scan; its last entry is the total)
    uint64_t* dist_scan = ensure<uint64_t>(c, B_DBG1, (n_tiles + 1) * 8);
    check(c, launch_scan_u32(s, tile_dist, n_tiles, dist_scan, scan_tmp), "scan");
    check(c, hipMemcpyAsync(h_binoff + gb1, dist_scan + n_tiles, 8, hipMemcpyDeviceToHost, s),
          "D2H");
    check(c, hipMemcpyAsync(h_misc_p, misc, sizeof(Misc), hipMemcpyDeviceToHost, s), "D2H");
    check(c, hipStreamSynchronize(s), "sync");
    big_tiles += h_misc_p->n_big;
    big_keys += h_misc_p->big_total;
    big_out += h_misc_p->big_out;
    };  // tile_pass

    if (kx) {
      // (k,x)-mers: the first pass sorts and counts the (k,x)-mers of the
      // records (every one kept); the second counts the k-mers of the
      // distinct (k,x)-mers, each weighted by its count, with the job's
      // cutoffs
      KeyCfg k1 = kc;
      k1.kx = kx;
      k1.kx_pass = 1;
      k1.cutoff_min = 1;
      k1.cutoff_max = 0xFFFFFFFFu;
      k1.counter_max = 0xFFFFFFFFu;
      tile_pass(grec, rs1.data(), rc1.data(), k1, false);
      for (int i = KMC_K_FINE_HIST; i <= KMC_K_BIG_TILES; ++i)
        kx_us[i] = 1e3 * ev_ms(c->ev[8 + 2 * i], c->ev[9 + 2 * i]);
      kx_us[KMC_K_ASSEMBLE] = 1e3 * ev_ms(c->ev[8 + 2 * KMC_K_ASSEMBLE],
                                          c->ev[9 + 2 * KMC_K_ASSEMBLE]);
      const uint64_t n1 = h_binoff[nbg];
      const std::vector<uint64_t> rs2(h_binoff, h_binoff + gb1);
      std::vector<uint64_t> rc2(nbg);
      for (uint32_t i = 0; i < nbg; ++i) rc2[i] = rs2[i + 1] - rs2[i];
      st.n_kx_distinct += n1;
      uint64_t* kxk = ensure<uint64_t>(c, B_KXK, std::max<uint64_t>(1, n1) * 8);
      uint32_t* kxc = ensure<uint32_t>(c, B_KXC, std::max<uint64_t>(1, n1) * 4);
      uint64_t* kxr = ensure<uint64_t>(c, B_KXR, std::max<uint64_t>(1, n1) * 16);
      uint64_t* kxs = ensure<uint64_t>(c, B_DBG2, (n1 + 1) * 8);
      uint64_t* kst = ensure<uint64_t>(c, B_SCANTMP,
                                       scan_tmp_words(std::max<uint64_t>(n_tiles, n1)) * 8);
      check(c, launch_gather(s, k1, tiles, n_tiles, tile_off, keys, counts, kxk, kxc),
            "gather (k,x)-mers");
      check(c, launch_scan_u32(s, kxc, n1, kxs, kst), "scan");
      check(c, launch_kx_records(s, kxk, kxc, n1, kxr), "(k,x)-mer records");
      uint64_t* h_kx = ensure_host<uint64_t>(c, H_KX, 8);
      check(c, hipMemcpyAsync(h_kx, kxs + n1, 8, hipMemcpyDeviceToHost, s), "D2H");
      check(c, hipMemsetAsync(misc, 0, sizeof(Misc), s), "memset");
      check(c, hipStreamSynchronize(s), "sync");
      st.n_kx_entries += *h_kx;
      KeyCfg k2 = kc;
      k2.kx = kx;
      k2.kx_pass = 2;
      tile_pass(kxr, rs2.data(), rc2.data(), k2, true);
    } else {
      tile_pass(grec, rs1.data(), rc1.data(), kc, false);
    }
    const uint64_t g_out = h_binoff[nbg];
    for (uint32_t i = 0; i <= nbg; ++i) T->bin_offsets[b0 + i] = n_out_total + h_binoff[i];
    n_distinct += h_binoff[gb1];
    if (!grouped) {
      // one group: the table is gathered straight into its final place
      n_out_total = g_out;
      break;
    }
    // a group of a grouped job: gathered into a staging block, appended to
    // the entries kept in host memory
    uint64_t* gk_out = ensure<uint64_t>(c, B_OUTK, std::max<uint64_t>(1, g_out) * J.kw * 8);
    uint32_t* gc_out = ensure<uint32_t>(c, B_OUTC, std::max<uint64_t>(1, g_out) * 4);
    check(c, hipEventRecord(c->ev[28], s), "event");
    check(c, launch_gather(s, kc, tiles, n_tiles, tile_off, keys, counts, gk_out, gc_out),
          "gather");
    check(c, hipEventRecord(c->ev[29], s), "event");
    // room for the whole table once the first group has shown its share
    // (groups hold about equal numbers of k-mers)
    if (!acc.reserve(std::max<uint64_t>(n_out_total + g_out,
                                        gi == 0 ? (g_out * groups.size() * 5) / 4 + 1 : 0),
                     n_out_total, J.kw)) {
      c->err = "host allocation of a grouped job's entries failed";
      throw Fail{KMC_ERR_OUT_OF_MEMORY};
    }
    if (g_out) {
      check(c, hipMemcpyAsync(acc.k + n_out_total * J.kw, gk_out, g_out * J.kw * 8,
                              hipMemcpyDeviceToHost, s), "D2H");
      check(c, hipMemcpyAsync(acc.c + n_out_total, gc_out, g_out * 4, hipMemcpyDeviceToHost,
                              s), "D2H");
    }
    check(c, hipStreamSynchronize(s), "sync");
    n_out_total += g_out;
    for (int i = KMC_K_FINE_HIST; i < KMC_N_KERNELS; ++i)
      acc_us[i] += 1e3 * ev_ms(c->ev[8 + 2 * i], c->ev[9 + 2 * i]);
    acc_us[KMC_K_ASSEMBLE] += 1e3 * ev_ms(c->ev[28], c->ev[29]);
    acc_phase[0] += 1e3 * ev_ms(gi == 0 ? c->ev[2] : c->ev[8 + 2 * KMC_K_FINE_HIST], c->ev[3]);
    acc_phase[1] += 1e3 * ev_ms(c->ev[3], c->ev[4]);
    acc_phase[2] += 1e3 * ev_ms(c->ev[4], c->ev[29]);
  }
  if (grouped) pool_next_group(c);  // every group's entries are in host memory
  st.n_tiles = n_tiles_all;
  st.n_big_tiles = big_tiles;
  st.n_big_keys = big_keys;
  st.n_big_out = big_out;
  const uint64_t n_out = n_out_total;
  st.n_out = n_out;
  st.n_distinct = n_distinct;
  T->n = n_out;
  // the table's keys and counts: the caller's buffers (allocation-free form),
  // the caller's workspace, a pooled device block, or host memory
  if (c->user_keys) {
    if (n_out > c->user_cap) {
      c->user_need = n_out;
      c->err = "the table has more entries than the output buffers hold";
      throw Fail{KMC_ERR_TOO_LARGE};
    }
    T->keys = c->user_keys;
    T->counts = c->user_counts;
    T->reserved = 1;
    out_k = T->keys;
    out_c = T->counts;
  } else if (T->on_device && c->ws_base && !c->ws_own_table) {
    // the table lives in the caller's workspace; kmc_table_free leaves it
    T->keys = ensure<uint64_t>(c, B_OUTK, n_out * J.kw * 8);
    T->counts = ensure<uint32_t>(c, B_OUTC, n_out * 4);
    T->reserved = 1;
    out_k = T->keys;
    out_c = T->counts;
  } else if (T->on_device || (grouped && (J.flags & KMC_FLAG_ASCENDING))) {
    // keys and counts in one pooled block
    const size_t kb = (std::max<uint64_t>(1, n_out * J.kw) * 8 + 255) & ~(size_t)255;
    void* blk = pool_take(c->device, kb + std::max<uint64_t>(1, n_out) * 4);
    if (!blk) {
      c->err = "device allocation of the table failed";
      throw Fail{KMC_ERR_OUT_OF_MEMORY};
    }
    T->keys = static_cast<uint64_t*>(blk);
    T->counts = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(blk) + kb);
    T->reserved = 2;
    T->on_device = 1;
    out_k = T->keys;
    out_c = T->counts;
  } else if (!grouped) {
    out_k = ensure<uint64_t>(c, B_OUTK, n_out * J.kw * 8);
    out_c = ensure<uint32_t>(c, B_OUTC, n_out * 4);
  }
  if (!grouped) {
    // the last (only) group's tiles are still in place: gather them
    check(c, hipEventRecord(c->ev[28], s), "event");
    const uint64_t n_tiles = n_tiles_all;
    check(c, launch_gather(s, kc, ensure<Tile>(c, B_TILES, n_tiles * sizeof(Tile)), n_tiles,
                           ensure<uint64_t>(c, B_TILEOFF, (n_tiles + 1) * 8),
                           ensure<uint64_t>(c, B_KEYS, n_kmers * J.kw * 8),
                           ensure<uint32_t>(c, B_COUNTS, n_kmers * 4), out_k, out_c),
          "gather");
  } else if (out_k && n_out) {
    // a grouped job's entries into the device table
    check(c, hipEventRecord(c->ev[28], s), "event");
    check(c, hipMemcpyAsync(out_k, acc.k, n_out * J.kw * 8, hipMemcpyHostToDevice, s),
          "H2D table");
    check(c, hipMemcpyAsync(out_c, acc.c, n_out * 4, hipMemcpyHostToDevice, s), "H2D table");
  } else {
    check(c, hipEventRecord(c->ev[28], s), "event");
  }
  if ((J.flags & KMC_FLAG_ASCENDING) && out_k) {
    // ascending over the whole table: segments by top key bits into a
    // scratch copy, groups ordered in LDS back into the table
    std::free(T->bin_offsets);
    T->bin_offsets = nullptr;
    if (n_out) {
      const AscPlan ap = plan_ascending(n_out, J.k, J.kw);
      const uint64_t nseg = 1ull << ap.seg_bits;
      auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
      const uint64_t o1 = al(nseg * 4), o2 = o1 + al((nseg + 1) * 8),
                     o3 = o2 + al(scan_tmp_words(nseg) * 8), o4 = o3 + (ap.n_groups + 1) * 8;
      uint8_t* sb = ensure<uint8_t>(c, B_ASCSEG, o4);
      uint64_t* xk = ensure<uint64_t>(c, B_ASCK, n_out * J.kw * 8);
      uint32_t* xc = ensure<uint32_t>(c, B_ASCC, n_out * 4);
      check(c, launch_ascending(s, kc, n_out, ap, reinterpret_cast<uint32_t*>(sb),
                                reinterpret_cast<uint64_t*>(sb + o1),
                                reinterpret_cast<uint64_t*>(sb + o2),
                                reinterpret_cast<uint64_t*>(sb + o3), xk, xc, out_k, out_c),
            "ascending");
    }
  }
  check(c, hipEventRecord(c->ev[29], s), "event");
  check(c, hipEventRecord(c->ev[5], s), "event");
  const bool want_host = !(J.flags & KMC_FLAG_DEVICE_TABLE) && !c->user_keys;
  if (want_host && grouped && !(J.flags & KMC_FLAG_ASCENDING)) {
    // a grouped job's host table: the memory that collected the entries
    T->on_device = 0;
    if (!acc.reserve(1, 0, J.kw)) {  // (a job without entries)
      c->err = "host allocation of the table failed";
      throw Fail{KMC_ERR_OUT_OF_MEMORY};
    }
    acc.give_to(T);
  } else if (want_host) {
    // a host table copied out of the device table (or the staging buffers)
    uint64_t* dk = out_k;
    uint32_t* dc = out_c;
    void* pooled = T->reserved == 2 ? T->keys : nullptr;
    T->on_device = 0;
    T->reserved = 0;
    T->keys = nullptr;
    T->counts = nullptr;
    try {
      host_table(T, n_out, J.kw);
    } catch (const Fail&) {
      if (pooled) pool_give(pooled);
      throw;
    }
    if (n_out) {
      check(c, hipMemcpyAsync(T->keys, dk, n_out * J.kw * 8, hipMemcpyDeviceToHost, s), "D2H");
      check(c, hipMemcpyAsync(T->counts, dc, n_out * 4, hipMemcpyDeviceToHost, s), "D2H");
    }
    check(c, hipStreamSynchronize(s), "sync");
    if (pooled) pool_give(pooled);
  }
  check(c, hipStreamSynchronize(s), "sync");
  st.us_map = 1e3 * ev_ms(c->ev[0], c->ev[1]);
  st.us_split = 1e3 * ev_ms(c->ev[1], c->ev[2]);
  st.us_total = 1e3 * ev_ms(c->ev[0], c->ev[5]);
  for (int i = 0; i < KMC_N_KERNELS; ++i)
    st.us_kernel[i] = 1e3 * ev_ms(c->ev[8 + 2 * i], c->ev[9 + 2 * i]);
  for (int i = 0; i < KMC_N_KERNELS; ++i) st.us_kernel[i] += kx_us[i];  // (k,x): first pass
  if (!grouped) {
    st.us_expand = 1e3 * ev_ms(c->ev[2], c->ev[3]);
    st.us_sort = 1e3 * ev_ms(c->ev[3], c->ev[4]);
    st.us_assemble = 1e3 * ev_ms(c->ev[4], c->ev[5]);
    st.us_kernel[KMC_K_ASSEMBLE] += 1e3 * ev_ms(c->ev[28], c->ev[29]);
  } else {
    for (int i = KMC_K_FINE_HIST; i < KMC_N_KERNELS; ++i) st.us_kernel[i] = acc_us[i];
    st.us_expand = acc_phase[0];
    st.us_sort = acc_phase[1];
    st.us_assemble = acc_phase[2];
  }
  // algorithmic bytes: input once, 2-bit payload of every super k-mer written
  // and read once (ceil(l/4) + 2 bytes each), keys written and read once,
  // output written once
  const uint64_t payload = n_rec * 2 + (n_kmers + n_rec * (J.k - 1)) / 4;
  st.bytes_alg = J.n_bases + 8 * (J.n_reads + 1) + 2 * payload +
                 2 * (uint64_t)(8 * J.kw) * n_kmers + (uint64_t)(8 * J.kw + 4) * n_out;
}

// Upper bounds of every buffer of one job, from its sizes alone: at most one
// k-mer per base, one record per k-mer (plus 256 per bin of sampling slack),
// every tile at most the LDS tile target, every tile possibly too big for LDS.
WsLayout plan_workspace(const kmc_reads* R, const kmc_params* P) {
  WsLayout L;
  const uint64_t N = R->n_bases, NR = R->n_reads, NB = P->n_bins;
  const uint64_t kw = P->k <= 32 ? 1 : 2, RW = 2 * kw;
  const uint64_t n_sig = (1ull << (2 * P->p)) + 1;
  const uint64_t kmax = N;
  const uint64_t recmax = kmax + 256 * NB;
  const uint64_t cap = kw == 1 ? kTileCap1 : kTileCap2, limit = 3 * cap / 4;
  const uint64_t tmax = 2 * (kmax / limit) + 3 * NB + 1;
  const uint64_t tasks = recmax / kExpandThreads + NB + 1;
  uint64_t sz[B_COUNT_] = {};
  sz[B_SEQ] = R->on_device ? 0 : N + 16;
  sz[B_OFF] = R->on_device ? 0 : (NR + 1) * 8;
  sz[B_HIST] = n_sig * 8;
  sz[B_MAP] = n_sig * 4;
  sz[B_BINCNT] = NB * 16;
  sz[B_CURSOR] = NB * 8;
  sz[B_REC] = recmax * RW * 8;
  // fine bits as the tile plan picks them, for a bin holding every k-mer
  const uint32_t fb = std::max<uint32_t>(
      1, std::min<uint32_t>({ilog2_ceil(kmax * 8 / cap + 1), (uint32_t)kMaxFineBits, 2 * P->k}));
  sz[B_FINE] = (NB << fb) * 4;
  sz[B_TOF] = (NB << fb) * 2;
  sz[B_TILES] = tmax * sizeof(Tile);
  sz[B_TCUR] = tmax * 8;
  sz[B_BASES] = 6 * (NB + 1) * 8;
  sz[B_HTASK] = tasks * sizeof(ExpandTask);
  sz[B_ETASK] = tasks * sizeof(ExpandTask);
  sz[B_KEYS] = kmax * kw * 8;
  sz[B_COUNTS] = kmax * 4;
  sz[B_TILEOUT] = tmax * 8 + 8;
  sz[B_BIG] = tmax * 20 + 16;
  sz[B_MISC] = sizeof(Misc);
  sz[B_TMP] = kmax * kw * 8;
  sz[B_SCANTMP] = scan_tmp_words(tmax) * 8;
  sz[B_TILEOFF] = (tmax + 1) * 8;
  sz[B_BINOFF] = (NB + 1) * 8;
  sz[B_OUTK] = kmax * kw * 8;
  sz[B_OUTC] = kmax * 4;
  sz[B_DBG1] = (tmax + 1) * 8;
  sz[B_DBG2] = 0;
  if (P->flags & KMC_FLAG_ASCENDING) {
    // ascending order: segment counters, offsets, scan scratch, group starts
    // (the plan for kmax entries has the most segments and groups), and a
    // scratch copy of the table
    const AscPlan ap = plan_ascending(kmax, P->k, (uint32_t)kw);
    const uint64_t nseg = 1ull << ap.seg_bits;
    sz[B_ASCSEG] = nseg * 4 + (nseg + 1) * 8 + scan_tmp_words(nseg) * 8 + (ap.n_groups + 1) * 8 +
                   4 * 256;
    sz[B_ASCK] = kmax * kw * 8;
    sz[B_ASCC] = kmax * 4;
  }
  // records are dead once the keys are expanded: the big-tile scratch and,
  // after it, the assembled table reuse their region
  auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  const uint64_t alias_tmp = sz[B_TMP], alias_k = sz[B_OUTK], alias_c = sz[B_OUTC];
  const uint64_t alias_xk = sz[B_ASCK], alias_xc = sz[B_ASCC];
  sz[B_TMP] = sz[B_OUTK] = sz[B_OUTC] = sz[B_ASCK] = sz[B_ASCC] = 0;
  sz[B_REC] = std::max<uint64_t>(
      {sz[B_REC], alias_tmp, al(alias_k) + al(alias_c) + al(alias_xk) + alias_xc});
  size_t at = 0;
  for (int i = 0; i < B_COUNT_; ++i) {
    L.off[i] = at;
    L.size[i] = (size_t)std::max<uint64_t>(sz[i], 16);
    at += al(L.size[i]);
  }
  L.off[B_TMP] = L.off[B_REC];
  L.size[B_TMP] = alias_tmp;
  L.off[B_OUTK] = L.off[B_REC];
  L.size[B_OUTK] = alias_k;
  L.off[B_OUTC] = L.off[B_REC] + al(alias_k);
  L.size[B_OUTC] = alias_c;
  // the ascending order's scratch copy follows the table (the big-tile
  // scratch is dead by then)
  L.off[B_ASCK] = L.off[B_OUTC] + al(alias_c);
  L.size[B_ASCK] = alias_xk;
  L.off[B_ASCC] = L.off[B_ASCK] + al(alias_xk);
  L.size[B_ASCC] = alias_xc;
  L.total = at;
  return L;
}

kmc_status guarded(kmc_ctx* c, const kmc_reads* R, const kmc_params* P, kmc_table** out) {
  kmc_table* T = new_table();
  if (!T) return KMC_ERR_OUT_OF_MEMORY;
  try {
    run_count(c, R, P, T);
  } catch (const Fail& f) {
    kmc_table_free(T);
    (void)hipStreamSynchronize(c->stream);
    return f.st;
  } catch (const std::bad_alloc&) {
    kmc_table_free(T);
    c->err = "host allocation failed";
    return KMC_ERR_OUT_OF_MEMORY;
  }
  *out = T;
  return KMC_OK;
}

thread_local kmc_ctx* t_default_ctx = nullptr;

}  // namespace

// ------------------------------------------------------------------- ABI

extern "C" {

kmc_status kmc_ctx_create(int device, kmc_ctx** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  kmc_ctx* c = new (std::nothrow) kmc_ctx();
  if (!c) return KMC_ERR_OUT_OF_MEMORY;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return KMC_ERR_DEVICE;
  }
  for (auto& e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      kmc_ctx_destroy(c);
      return KMC_ERR_DEVICE;
    }
  }
  *out = c;
  return KMC_OK;
}

void kmc_ctx_destroy(kmc_ctx* c) {
  if (!c) return;
  if (c->ext && c->ext_free) c->ext_free(c->ext);
  c->ext = nullptr;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->buf)
    if (b.p) (void)hipFree(b.p);
  for (auto& b : c->hbuf)
    if (b.p) (void)hipHostFree(b.p);
  if (c->spill.p) (void)hipHostFree(c->spill.p);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* kmc_last_error(const kmc_ctx* c) { return c ? c->err.c_str() : ""; }

kmc_status kmc_ctx_set_budget(kmc_ctx* c, uint64_t device_bytes) {
  if (!c) return KMC_ERR_INVALID_ARG;
  c->budget = device_bytes;
  return KMC_OK;
}

kmc_status kmc_ctx_set_knobs(kmc_ctx* c, const kmc_knobs* knobs) {
  if (!c) return KMC_ERR_INVALID_ARG;
  if (!knobs) {
    c->has_knobs = false;
    return KMC_OK;
  }
  if ((knobs->tile_fill != 0 && knobs->tile_fill != 2 && knobs->tile_fill != 3) ||
      knobs->fine_bits_bias < -2 || knobs->fine_bits_bias > 2 ||
      (knobs->expand_task != 0 && knobs->expand_task != 256 && knobs->expand_task != 512 &&
       knobs->expand_task != 1024))
    return KMC_ERR_INVALID_ARG;
  c->knobs = *knobs;
  c->has_knobs = true;
  return KMC_OK;
}

const char* kmc_status_str(kmc_status st) {
  switch (st) {
    case KMC_OK: return "ok";
    case KMC_ERR_INVALID_ARG: return "invalid argument";
    case KMC_ERR_OUT_OF_MEMORY: return "out of memory";
    case KMC_ERR_DEVICE: return "device error";
    case KMC_ERR_TOO_LARGE: return "job too large";
    case KMC_ERR_BUSY: return "busy";
  }
  return "unknown status";
}

}  // extern "C"

// Extension slot of a context (used by the batch worker pool).
void** kmc::ctx_ext(kmc_ctx* c, void (*release)(void*)) {
  if (release) c->ext_free = release;
  return &c->ext;
}
int kmc::ctx_device(const kmc_ctx* c) { return c->device; }
hipStream_t kmc::ctx_stream(const kmc_ctx* c) { return c->stream; }
void kmc::ctx_set_error(kmc_ctx* c, const char* msg) { c->err = msg ? msg : ""; }
void kmc::ctx_release_buffers(kmc_ctx* c) {
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->buf) {
    if (b.p && !c->pool_base) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  if (c->spill.p) (void)hipHostFree(c->spill.p);
  c->spill.p = nullptr;
  c->spill.cap = 0;
}
void kmc::ctx_set_budget(kmc_ctx* c, uint64_t bytes) { c->budget = bytes; }
void kmc::ctx_lend_region(kmc_ctx* c, void* base, size_t bytes) {
  kmc::ctx_release_buffers(c);
  c->pool_base = static_cast<uint8_t*>(base);
  c->pool_bytes = bytes;
  c->pool_top = c->pool_mark = 0;
}
void kmc::ctx_end_region(kmc_ctx* c) {
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->buf) b = DevBuf{};  // inside the lent region: not freed here
  c->pool_base = nullptr;
  c->pool_bytes = c->pool_top = c->pool_mark = 0;
}
void kmc::ctx_copy_tuning(kmc_ctx* dst, const kmc_ctx* src) {
  dst->has_knobs = src->has_knobs;
  dst->knobs = src->knobs;
  dst->tuned = src->tuned;
}
void kmc::ctx_set_tuned(kmc_ctx* c, uint32_t key_words, uint64_t n_bases, const kmc_knobs& k) {
  c->tuned[job_class(key_words, n_bases)] = k;
}
uint32_t kmc::ctx_batch_workers(const kmc_ctx* c) { return c->batch_workers; }
void kmc::ctx_set_batch_workers(kmc_ctx* c, uint32_t n) { c->batch_workers = n; }
bool kmc::ctx_override_knobs(kmc_ctx* c, const kmc_knobs* k) {
  const bool had = c->has_knobs;
  if (k) {
    c->knobs = *k;
    c->has_knobs = true;
  } else {
    c->has_knobs = false;
  }
  return had;
}
void* kmc::ctx_aux_buffer(kmc_ctx* c, int slot, size_t bytes) {
  if (slot < 0 || slot >= kCtxAuxBuffers) return nullptr;
  uint8_t* saved = c->ws_base;
  c->ws_base = nullptr;  // always the context's own cached buffers
  void* p = nullptr;
  try {
    p = ensure<uint8_t>(c, static_cast<BufId>(B_AUX0 + slot), bytes);
  } catch (const Fail&) {
    p = nullptr;
  }
  c->ws_base = saved;
  return p;
}

extern "C" {

kmc_status kmc_count_ex(kmc_ctx* c, const kmc_reads* reads, const kmc_params* params,
                        void* stream, kmc_table** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!c) return KMC_ERR_INVALID_ARG;
  c->err.clear();
  kmc_status v = validate(reads, params);
  if (v != KMC_OK) {
    c->err = "argument validation failed";
    return v;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  hipStream_t saved = c->stream;
  if (stream) c->stream = static_cast<hipStream_t>(stream);
  kmc_status st = guarded(c, reads, params, out);
  c->stream = saved;
  return st;
}

kmc_status kmc_count(const kmc_reads* reads, uint32_t k, uint32_t p, uint32_t n_bins,
                     uint32_t cutoff_min, uint32_t cutoff_max, kmc_table** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  kmc_params P{k, p, n_bins, cutoff_min, cutoff_max, 0, 0};
  kmc_status v = validate(reads, &P);  // before any device work
  if (v != KMC_OK) return v;
  if (!t_default_ctx) {
    kmc_status st = kmc_ctx_create(0, &t_default_ctx);
    if (st != KMC_OK) return st;
  }
  return kmc_count_ex(t_default_ctx, reads, &P, nullptr, out);
}

void kmc_table_free(kmc_table* t) {
  if (!t) return;
  if (t->on_device && t->reserved == 1) {
    // keys/counts belong to a caller's workspace
  } else if (t->on_device && t->reserved == 2) {
    if (t->keys && !pool_give(t->keys)) (void)hipFree(t->keys);
  } else if (t->on_device) {
    if (t->keys) (void)hipFree(t->keys);
    if (t->counts) (void)hipFree(t->counts);
  } else if (t->reserved == 3) {
    if (t->keys) pool_give(t->keys);  // pinned host block, back to the pool
  } else {
    std::free(t->keys);
    std::free(t->counts);
  }
  std::free(t->bin_offsets);
  std::free(t->sig_to_bin);
  std::free(t);
}

kmc_status kmc_workspace_size(const kmc_reads* reads, const kmc_params* params, size_t* bytes) {
  if (!bytes) return KMC_ERR_INVALID_ARG;
  *bytes = 0;
  kmc_status v = validate(reads, params);
  if (v != KMC_OK) return v;
  *bytes = plan_workspace(reads, params).total;
  return KMC_OK;
}

kmc_status kmc_count_ws(kmc_ctx* c, const kmc_reads* reads, const kmc_params* params,
                        void* stream, void* workspace, size_t ws_bytes, kmc_table** out) {
  return kmc::count_ws_impl(c, reads, params, stream, workspace, ws_bytes, false, out);
}

}  // extern "C"

kmc_status kmc::count_ws_impl(kmc_ctx* c, const kmc_reads* reads, const kmc_params* params,
                              void* stream, void* workspace, size_t ws_bytes, bool own_table,
                              kmc_table** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!c || !workspace || ((uintptr_t)workspace & 255u)) return KMC_ERR_INVALID_ARG;
  c->err.clear();
  kmc_status v = validate(reads, params);
  if (v != KMC_OK) {
    c->err = "argument validation failed";
    return v;
  }
  const WsLayout L = plan_workspace(reads, params);
  if (ws_bytes < L.total) {
    c->err = "workspace smaller than kmc_workspace_size";
    return KMC_ERR_OUT_OF_MEMORY;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  hipStream_t saved = c->stream;
  if (stream) c->stream = static_cast<hipStream_t>(stream);
  c->ws_base = static_cast<uint8_t*>(workspace);
  c->ws = L;
  c->ws_own_table = own_table;
  kmc_status st = guarded(c, reads, params, out);
  c->ws_base = nullptr;
  c->ws_own_table = false;
  c->stream = saved;
  return st;
}

kmc_status kmc::count_static_impl(kmc_ctx* c, const kmc_reads* reads, const kmc_params* params,
                                  void* stream, void* scratch, size_t scratch_bytes,
                                  uint64_t* keys_out, uint32_t* counts_out, uint64_t out_cap,
                                  uint64_t* n_out, uint64_t* bin_offsets, kmc_stats* stats) {
  if (!c || !n_out || !scratch || ((uintptr_t)scratch & 255u)) return KMC_ERR_INVALID_ARG;
  *n_out = 0;
  if (out_cap > 0 && (!keys_out || !counts_out)) return KMC_ERR_INVALID_ARG;
  c->err.clear();
  kmc_status v = validate(reads, params);
  if (v != KMC_OK) {
    c->err = "argument validation failed";
    return v;
  }
  const WsLayout L = plan_workspace(reads, params);
  if (L.total > scratch_bytes) {
    c->err = "the job needs " + std::to_string(L.total) + " bytes of scratch; the static scratch holds " +
             std::to_string(scratch_bytes);
    return KMC_ERR_TOO_LARGE;
  }
  hipStream_t saved = c->stream;
  if (stream) c->stream = static_cast<hipStream_t>(stream);
  c->ws_base = static_cast<uint8_t*>(scratch);
  c->ws = L;
  c->pageable_host = true;
  // a dummy 16-byte-aligned address keeps the caller-buffer branch taken for
  // an empty output
  static uint64_t empty_out[2];
  c->user_keys = keys_out ? keys_out : empty_out;
  c->user_counts = counts_out ? counts_out : reinterpret_cast<uint32_t*>(empty_out);
  c->user_cap = out_cap;
  c->user_need = 0;
  kmc_params P = *params;
  P.flags |= KMC_FLAG_DEVICE_TABLE;
  kmc_table* T = nullptr;
  kmc_status st = guarded(c, reads, &P, &T);
  c->ws_base = nullptr;
  c->pageable_host = false;
  c->user_keys = nullptr;
  c->user_counts = nullptr;
  c->user_cap = 0;
  c->stream = saved;
  if (st != KMC_OK) {
    if (st == KMC_ERR_TOO_LARGE) *n_out = c->user_need;
    return st;
  }
  *n_out = T->n;
  if (bin_offsets && T->bin_offsets)
    std::memcpy(bin_offsets, T->bin_offsets, ((size_t)T->n_bins + 1) * 8);
  if (stats) *stats = T->stats;
  kmc_table_free(T);  // host parts only: keys/counts are the caller's
  return KMC_OK;
}

extern "C" {

kmc_status kmc_debug_signatures(kmc_ctx* c, const kmc_reads* reads, uint32_t k, uint32_t p,
                                uint32_t flags, uint32_t* sig_per_window,
                                uint8_t* superkmer_start) {
  if (!c || !sig_per_window) return KMC_ERR_INVALID_ARG;
  kmc_params P{k, p, 1, 1, 1, flags & KMC_FLAG_PLAIN_MINIMIZERS, 0};
  kmc_status v = validate(reads, &P);
  if (v != KMC_OK) return v;
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  try {
    Job J;
    J.k = k;
    J.p = p;
    J.n_bins = 1;
    J.ci = J.cx = 1;
    J.kw = k <= 32 ? 1 : 2;
    J.flags = P.flags;
    stage_reads(c, reads, J);
    const ScanCfg C = scan_cfg(J);
    uint32_t* sig = ensure<uint32_t>(c, B_DBG1, J.n_bases * 4);
    uint8_t* st = ensure<uint8_t>(c, B_DBG2, J.n_bases);
    check(c, hipMemsetAsync(sig, 0xFF, J.n_bases * 4, c->stream), "memset");
    check(c, hipMemsetAsync(st, 0, J.n_bases, c->stream), "memset");
    check(c, launch_debug_sigs(c->stream, J.seq, J.off, J.n_reads, J.n_bases, C, J.kw, sig, st),
          "debug_sigs");
    if (J.n_bases) {
      check(c, hipMemcpyAsync(sig_per_window, sig, J.n_bases * 4, hipMemcpyDeviceToHost, c->stream), "D2H");
      if (superkmer_start)
        check(c, hipMemcpyAsync(superkmer_start, st, J.n_bases, hipMemcpyDeviceToHost, c->stream), "D2H");
    }
    check(c, hipStreamSynchronize(c->stream), "sync");
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(c->stream);
    return f.st;
  }
  return KMC_OK;
}

}  // extern "C"
