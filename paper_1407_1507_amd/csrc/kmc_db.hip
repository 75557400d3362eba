// The KMC 2 database layout (supplement, "Database format") built on the
// device from a counted table, written to and read from the .kmc_pre /
// .kmc_suf files, and queried in batches on the device (the random-access
// lookup of the supplement's API: CheckKmer), or decoded back into a table
// (the API's listing, ReadNextKmer, for every k-mer at once).
//
// Layout (all on the device):
//   map       uint32[4^p + 1]: prefix array of every signature value (the
//             table's signature -> bin map; the last entry is for k-mers with
//             no allowed p-mer);
//   prefixes  n_bins arrays of 4^lut uint64, then one guard: entry x of array
//             b is the index of the first record whose k-mer lies in bin b and
//             begins with the lut-symbol prefix x (the guard is the number of
//             records), so the records of (b, x) are [pre[x], pre[x + 1]);
//   records   the table's entries in its order (bin by bin, ascending keys
//             inside a bin): the k - lut symbols after the prefix packed four
//             to a byte, leftmost symbol first and in the byte's high bits,
//             then the count on counter_size bytes, least significant first.
// A lookup takes the k-mer's signature -> map -> prefix array, its prefix ->
// a record range, and a binary search of its suffix in that range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/kmc.h"
#include "kmc_device.h"
#include "kmc_internal.h"

using namespace kmc;

struct kmc_db {
  int device = 0;
  kmc_db_info info{};
  uint32_t n_bins = 0;
  uint32_t suf_bytes = 0, rec_bytes = 0;
  uint32_t* map = nullptr;   // device, 4^p + 1
  uint64_t* pre = nullptr;   // device, n_bins * 4^lut + 1
  uint8_t* rec = nullptr;    // device, total * rec_bytes
};

namespace {

constexpr uint32_t kDbVersion = 0x200;    // the KMC_VER field of a KMC 2 database
constexpr uint64_t kMaxPrefixEntries = 1ull << 28;  // n_bins * 4^lut (2 GiB of uint64)

template <int KW>
__device__ __forceinline__ typename KeyOf<KW>::T key_at(const uint64_t* keys, uint64_t i) {
  if constexpr (KW == 1) {
    return keys[i];
  } else {
    return ((u128)keys[2 * i] << 64) | keys[2 * i + 1];
  }
}

// Signature of a packed k-mer: the smallest allowed canonical p-mer in it
// (Methods, "From minimizers to signatures"); every canonical p-mer with
// filter == 0 (plain minimizers); 4^p when none is allowed.
template <class K>
__device__ uint32_t key_signature(K key, uint32_t k, uint32_t p, bool filter) {
  const uint32_t pmask = (1u << (2 * p)) - 1u;
  uint32_t best = 1u << (2 * p);
  for (uint32_t j = 0; j + p <= k; ++j) {
    const uint32_t f = (uint32_t)(key >> (2 * (k - p - j))) & pmask;
    const uint32_t r = (uint32_t)revcomp64((uint64_t)f, p);
    const uint32_t c = min(f, r);
    if (!filter || sig_allowed(c, p)) best = min(best, c);
  }
  return best;
}

// Suffix (the low 2(k - lut) bits of the key) of record r, read from its
// suf_bytes bytes (leftmost symbol first).
template <int KW>
__device__ __forceinline__ typename KeyOf<KW>::T read_suffix(const uint8_t* rec, uint32_t sb) {
  typedef typename KeyOf<KW>::T K;
  K v = 0;
  for (uint32_t j = 0; j < sb; ++j) v = (v << 8) | (K)rec[j];
  return v;
}

// The same from aligned 8-byte words of the records (the record buffer is
// padded by kRecPad bytes, so the words of the last record stay inside it):
// one load per word instead of one per byte.
constexpr size_t kRecPad = 32;
template <int KW>
__device__ __forceinline__ typename KeyOf<KW>::T read_suffix_words(const uint8_t* recs, uint64_t a,
                                                                   uint32_t sb) {
  typedef typename KeyOf<KW>::T K;
  if (sb == 0) return 0;
  const uint64_t* w = reinterpret_cast<const uint64_t*>(recs) + (a >> 3);
  const uint32_t s = 8 * (uint32_t)(a & 7);
  // bytes a .. a + 7 (and a + 8 .. a + 15), first byte lowest
  const uint64_t w0 = w[0], w1 = w[1];
  const uint64_t b0 = s ? (w0 >> s) | (w1 << (64 - s)) : w0;
  if constexpr (KW == 1) {
    return __builtin_bswap64(b0) >> (8 * (8 - sb));
  } else {
    const uint64_t w2 = sb + (a & 7) > 16 ? w[2] : 0;
    const uint64_t b1 = s ? (w1 >> s) | (w2 << (64 - s)) : w1;
    const K v = ((K)__builtin_bswap64(b0) << 64) | (K)__builtin_bswap64(b1);
    return v >> (8 * (16 - sb));
  }
}

__device__ __forceinline__ uint32_t read_count(const uint8_t* c, uint32_t cs) {
  uint32_t v = 0;
  for (uint32_t j = 0; j < cs; ++j) v |= (uint32_t)c[j] << (8 * j);
  return v;
}

// pre[b * L + x] = first entry of bin b whose prefix is >= x (a lower bound
// over the bin's ascending keys); the last thread writes the guard.
template <int KW>
__global__ void __launch_bounds__(256)
k_db_prefix(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ bo, uint32_t n_bins,
            uint32_t k, uint32_t lut, uint64_t* pre) {
  const uint64_t L = 1ull << (2 * lut);
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx > (uint64_t)n_bins * L) return;
  if (idx == (uint64_t)n_bins * L) {
    pre[idx] = bo[n_bins];
    return;
  }
  const uint32_t b = (uint32_t)(idx / L);
  const uint64_t x = idx % L;
  uint64_t lo = bo[b], hi = bo[b + 1];
  const uint32_t sh = 2 * (k - lut);
  while (lut && lo < hi) {  // with no prefix symbols every record starts its bin
    const uint64_t mid = (lo + hi) >> 1;
    if ((uint64_t)(key_at<KW>(keys, mid) >> sh) < x) lo = mid + 1;
    else hi = mid;
  }
  pre[idx] = lo;
}

// Record of every entry: suffix bytes, then the count clipped to the counter
// field, least significant byte first.
template <int KW>
__global__ void __launch_bounds__(256)
k_db_records(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ counts, uint64_t n,
             uint32_t sb, uint32_t cs, uint8_t* out) {
  typedef typename KeyOf<KW>::T K;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const K key = key_at<KW>(keys, i);
  uint8_t* r = out + i * (sb + cs);
  for (uint32_t j = 0; j < sb; ++j) r[j] = (uint8_t)(key >> (8 * (sb - 1 - j)));
  const uint32_t cmax = cs >= 4 ? 0xFFFFFFFFu : (1u << (8 * cs)) - 1u;
  const uint32_t c = min(counts[i], cmax);
  for (uint32_t j = 0; j < cs; ++j) r[sb + j] = (uint8_t)(c >> (8 * j));
}

struct DbView {
  const uint32_t* map;
  const uint64_t* pre;
  const uint8_t* rec;
  uint32_t k, p, lut, sb, cs, canonical, filter;
};

// Count of every query k-mer (packed as read): canonical form when the
// database is canonical, signature -> prefix array, prefix -> record range,
// binary search of the suffix; 0 when absent or outside [cmin, cmax].
template <int KW>
__global__ void __launch_bounds__(256)
k_db_query(DbView D, const uint64_t* __restrict__ q, uint64_t n, uint32_t cmin, uint32_t cmax,
           uint32_t* out) {
  typedef typename KeyOf<KW>::T K;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const K kmask = key_mask<K>(D.k);
  K key = key_at<KW>(q, i) & kmask;
  if (D.canonical) {
    const K rc = revcomp_key(key, D.k);
    key = rc < key ? rc : key;
  }
  const uint32_t sig = key_signature(key, D.k, D.p, D.filter != 0);
  const uint64_t L = 1ull << (2 * D.lut);
  const uint32_t sh = 2 * (D.k - D.lut);
  const uint64_t x = D.lut ? (uint64_t)(key >> sh) : 0;
  const K suf = sh >= 8 * sizeof(K) ? key : (key & ((K(1) << sh) - 1));
  const uint64_t slot = (uint64_t)D.map[sig] * L + x;
  uint64_t lo = D.pre[slot], hi = D.pre[slot + 1];
  const uint32_t rb = D.sb + D.cs;
  uint32_t c = 0;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    const K v = read_suffix_words<KW>(D.rec, mid * rb, D.sb);
    if (v == suf) {
      c = read_count(D.rec + mid * rb + D.sb, D.cs);
      break;
    }
    if (v < suf) lo = mid + 1;
    else hi = mid;
  }
  out[i] = (c >= cmin && c <= cmax) ? c : 0u;
}

// Every record back into (key, count): its prefix array and prefix from an
// upper bound over the prefix entries, its suffix from its bytes.
template <int KW>
__global__ void __launch_bounds__(256)
k_db_decode(DbView D, uint64_t n_slots, uint64_t n, uint64_t* keys, uint32_t* counts) {
  typedef typename KeyOf<KW>::T K;
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  // the last slot s with pre[s] <= r
  uint64_t lo = 0, hi = n_slots;  // pre[0] == 0 <= r
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (D.pre[mid] <= r) lo = mid;
    else hi = mid;
  }
  const uint64_t L = 1ull << (2 * D.lut);
  const uint64_t x = lo % L;
  const uint32_t rb = D.sb + D.cs;
  const K suf = read_suffix<KW>(D.rec + r * rb, D.sb);
  const uint32_t sh = 2 * (D.k - D.lut);
  const K key = D.lut ? (((K)x << sh) | suf) : suf;
  if constexpr (KW == 1) {
    keys[r] = key;
  } else {
    keys[2 * r] = (uint64_t)(key >> 64);
    keys[2 * r + 1] = (uint64_t)key;
  }
  counts[r] = read_count(D.rec + r * rb + D.sb, D.cs);
}

DbView view(const kmc_db* db) {
  DbView D;
  D.map = db->map;
  D.pre = db->pre;
  D.rec = db->rec;
  D.k = db->info.kmer_length;
  D.p = db->info.signature_length;
  D.lut = db->info.lut_prefix_length;
  D.sb = db->suf_bytes;
  D.cs = db->info.counter_size;
  D.canonical = (db->info.flags & KMC_FLAG_NON_CANONICAL) ? 0u : 1u;
  D.filter = (db->info.flags & KMC_FLAG_PLAIN_MINIMIZERS) ? 0u : 1u;
  return D;
}

uint32_t grid(uint64_t n) { return (uint32_t)((n + 255) / 256); }

void free_parts(kmc_db* db) {
  if (!db) return;
  (void)hipSetDevice(db->device);
  if (db->map) (void)hipFree(db->map);
  if (db->pre) (void)hipFree(db->pre);
  if (db->rec) (void)hipFree(db->rec);
  delete db;
}

// Sizes of a database from its parameters; false if they are out of range.
bool shape(kmc_db* db, std::string& why) {
  const kmc_db_info& I = db->info;
  if (I.kmer_length < 4 || I.kmer_length > 64 || I.signature_length < 4 ||
      I.signature_length > 12 || I.signature_length > I.kmer_length) {
    why = "k or p out of range";
    return false;
  }
  if (I.lut_prefix_length > I.kmer_length || (I.kmer_length - I.lut_prefix_length) % 4 != 0) {
    why = "4 must divide kmer_length - lut_prefix_length";
    return false;
  }
  if (I.counter_size < 1 || I.counter_size > 4) {
    why = "counter_size must be 1..4";
    return false;
  }
  if (I.lut_prefix_length > 14 ||
      (uint64_t)db->n_bins * (1ull << (2 * I.lut_prefix_length)) > kMaxPrefixEntries) {
    why = "n_bins * 4^lut_prefix_length above 2^28 prefix entries";
    return false;
  }
  db->suf_bytes = (I.kmer_length - I.lut_prefix_length) / 4;
  db->rec_bytes = db->suf_bytes + I.counter_size;
  return true;
}

template <class T>
bool dev_alloc(T** p, size_t n) {
  if (hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}

void put32(std::vector<uint8_t>& v, uint32_t x) {
  for (int i = 0; i < 4; ++i) v.push_back((uint8_t)(x >> (8 * i)));
}
void put64(std::vector<uint8_t>& v, uint64_t x) {
  for (int i = 0; i < 8; ++i) v.push_back((uint8_t)(x >> (8 * i)));
}
uint32_t get32(const uint8_t* p) {
  return (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24;
}
uint64_t get64(const uint8_t* p) { return (uint64_t)get32(p) | (uint64_t)get32(p + 4) << 32; }

bool read_file(const std::string& path, std::vector<uint8_t>& out) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  bool ok = std::fseek(f, 0, SEEK_END) == 0;
  const long n = ok ? std::ftell(f) : -1;
  ok = ok && n >= 0 && std::fseek(f, 0, SEEK_SET) == 0;
  if (ok) {
    out.resize((size_t)n);
    ok = n == 0 || std::fread(out.data(), 1, (size_t)n, f) == (size_t)n;
  }
  std::fclose(f);
  return ok;
}

bool write_file(const std::string& path, const std::vector<uint8_t>& a, const uint8_t* b,
                size_t nb, const std::vector<uint8_t>& c) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) return false;
  bool ok = std::fwrite(a.data(), 1, a.size(), f) == a.size();
  ok = ok && (nb == 0 || std::fwrite(b, 1, nb, f) == nb);
  ok = ok && std::fwrite(c.data(), 1, c.size(), f) == c.size();
  return std::fclose(f) == 0 && ok;
}

}  // namespace

extern "C" {

kmc_status kmc_db_build(kmc_ctx* ctx, const kmc_table* table, const kmc_params* params,
                        uint32_t lut_prefix_len, uint32_t counter_size, kmc_db** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!ctx || !table || !params || !table->bin_offsets || !table->sig_to_bin)
    return KMC_ERR_INVALID_ARG;
  if (params->k != table->k || params->p != table->p || params->n_bins != table->n_bins)
    return KMC_ERR_INVALID_ARG;
  kmc_db* db = new (std::nothrow) kmc_db();
  if (!db) return KMC_ERR_OUT_OF_MEMORY;
  db->device = ctx_device(ctx);
  db->n_bins = table->n_bins;
  kmc_db_info& I = db->info;
  I.kmer_length = table->k;
  I.mode = 0;
  I.counter_size = counter_size;
  I.lut_prefix_length = lut_prefix_len;
  I.signature_length = table->p;
  I.min_count = params->cutoff_min == 0 ? 1 : params->cutoff_min;
  I.max_count = params->cutoff_max;
  I.total_kmers = table->n;
  I.flags = params->flags & (KMC_FLAG_NON_CANONICAL | KMC_FLAG_PLAIN_MINIMIZERS);
  std::string why;
  if (!shape(db, why)) {
    ctx_set_error(ctx, why.c_str());
    delete db;
    return KMC_ERR_INVALID_ARG;
  }
  if (hipSetDevice(db->device) != hipSuccess) {
    (void)hipGetLastError();
    delete db;
    return KMC_ERR_DEVICE;
  }
  const uint32_t kw = table->key_words;
  const uint64_t n = table->n, L = 1ull << (2 * lut_prefix_len);
  const uint64_t n_sig = (1ull << (2 * table->p)) + 1;
  const uint64_t n_pre = (uint64_t)db->n_bins * L + 1;
  hipStream_t s = ctx_stream(ctx);
  const uint64_t* keys = table->keys;
  const uint32_t* counts = table->counts;
  uint64_t* tk = nullptr;
  uint32_t* tc = nullptr;
  uint64_t* bo = nullptr;
  kmc_status st = KMC_OK;
  auto fail = [&](kmc_status e, const char* what) {
    ctx_set_error(ctx, what);
    st = e;
  };
  do {
    if (!dev_alloc(&db->map, n_sig) || !dev_alloc(&db->pre, n_pre) ||
        !dev_alloc(&db->rec, n * db->rec_bytes + kRecPad) || !dev_alloc(&bo, db->n_bins + 1)) {
      fail(KMC_ERR_OUT_OF_MEMORY, "device allocation of the database failed");
      break;
    }
    if (!table->on_device && n) {
      // host table: staged on the device for the build
      if (!dev_alloc(&tk, n * kw) || !dev_alloc(&tc, n)) {
        fail(KMC_ERR_OUT_OF_MEMORY, "device allocation of the staged table failed");
        break;
      }
      if (hipMemcpyAsync(tk, table->keys, n * kw * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(tc, table->counts, n * 4, hipMemcpyHostToDevice, s) != hipSuccess) {
        fail(KMC_ERR_DEVICE, "H2D of the table failed");
        break;
      }
      keys = tk;
      counts = tc;
    }
    if (hipMemcpyAsync(db->map, table->sig_to_bin, n_sig * 4, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(bo, table->bin_offsets, (db->n_bins + 1) * 8, hipMemcpyHostToDevice, s) !=
            hipSuccess) {
      fail(KMC_ERR_DEVICE, "H2D of the map failed");
      break;
    }
    if (kw == 1) {
      hipLaunchKernelGGL(k_db_prefix<1>, dim3(grid(n_pre)), dim3(256), 0, s, keys, bo,
                         db->n_bins, I.kmer_length, lut_prefix_len, db->pre);
      if (n)
        hipLaunchKernelGGL(k_db_records<1>, dim3(grid(n)), dim3(256), 0, s, keys, counts, n,
                           db->suf_bytes, counter_size, db->rec);
    } else {
      hipLaunchKernelGGL(k_db_prefix<2>, dim3(grid(n_pre)), dim3(256), 0, s, keys, bo,
                         db->n_bins, I.kmer_length, lut_prefix_len, db->pre);
      if (n)
        hipLaunchKernelGGL(k_db_records<2>, dim3(grid(n)), dim3(256), 0, s, keys, counts, n,
                           db->suf_bytes, counter_size, db->rec);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      fail(KMC_ERR_DEVICE, "database build kernels failed");
      break;
    }
  } while (false);
  if (tk) (void)hipFree(tk);
  if (tc) (void)hipFree(tc);
  if (bo) (void)hipFree(bo);
  if (st != KMC_OK) {
    free_parts(db);
    return st;
  }
  *out = db;
  return KMC_OK;
}

kmc_status kmc_db_info_get(const kmc_db* db, kmc_db_info* info) {
  if (!db || !info) return KMC_ERR_INVALID_ARG;
  *info = db->info;
  return KMC_OK;
}

kmc_status kmc_db_write(const kmc_db* db, const char* path_prefix) {
  if (!db || !path_prefix) return KMC_ERR_INVALID_ARG;
  if (hipSetDevice(db->device) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  const kmc_db_info& I = db->info;
  const uint64_t L = 1ull << (2 * I.lut_prefix_length);
  const uint64_t n_pre = (uint64_t)db->n_bins * L + 1;
  const uint64_t n_sig = (1ull << (2 * I.signature_length)) + 1;
  const uint64_t nrec = I.total_kmers * db->rec_bytes;
  std::vector<uint64_t> pre(n_pre);
  std::vector<uint32_t> map(n_sig);
  std::vector<uint8_t> rec(nrec);
  if (hipMemcpy(pre.data(), db->pre, n_pre * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(map.data(), db->map, n_sig * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      (nrec && hipMemcpy(rec.data(), db->rec, nrec, hipMemcpyDeviceToHost) != hipSuccess)) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  // .kmc_pre: marker, prefixes (+ guard), map, header, header position, marker
  std::vector<uint8_t> head;
  head.insert(head.end(), {'K', 'M', 'C', 'P'});
  head.reserve(4 + n_pre * 8 + n_sig * 4 + 128);
  for (uint64_t v : pre) put64(head, v);
  for (uint32_t v : map) put32(head, v);
  const size_t h0 = head.size();
  put32(head, I.kmer_length);
  put32(head, I.mode);
  put32(head, I.counter_size);
  put32(head, I.lut_prefix_length);
  put32(head, I.signature_length);
  put32(head, I.min_count);
  put32(head, I.max_count);
  put64(head, I.total_kmers);
  // tmp[7] (unused by the format): tmp[0] records the counting variant
  // (plain minimizers, k-mers as read), 0 for the paper's own database
  put32(head, I.flags);
  for (int i = 1; i < 7; ++i) put32(head, 0);
  put32(head, kDbVersion);
  const uint32_t hlen = (uint32_t)(head.size() - h0);
  put32(head, hlen);
  head.insert(head.end(), {'K', 'M', 'C', 'P'});
  const std::string base(path_prefix);
  const std::vector<uint8_t> none;
  if (!write_file(base + ".kmc_pre", head, nullptr, 0, none)) return KMC_ERR_INVALID_ARG;
  const std::vector<uint8_t> ms = {'K', 'M', 'C', 'S'};
  if (!write_file(base + ".kmc_suf", ms, rec.data(), rec.size(), ms)) return KMC_ERR_INVALID_ARG;
  return KMC_OK;
}

kmc_status kmc_db_open(kmc_ctx* ctx, const char* path_prefix, kmc_db** out) {
  if (!out) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!ctx || !path_prefix) return KMC_ERR_INVALID_ARG;
  const std::string base(path_prefix);
  std::vector<uint8_t> pf, sf;
  if (!read_file(base + ".kmc_pre", pf) || !read_file(base + ".kmc_suf", sf)) {
    ctx_set_error(ctx, "cannot read the database files");
    return KMC_ERR_INVALID_ARG;
  }
  auto marker = [](const std::vector<uint8_t>& v, size_t at, const char* m) {
    return at + 4 <= v.size() && std::memcmp(v.data() + at, m, 4) == 0;
  };
  // markers at both ends, the header position 8 bytes from the end, the
  // header that many bytes before it
  if (pf.size() < 16 || !marker(pf, 0, "KMCP") || !marker(pf, pf.size() - 4, "KMCP") ||
      sf.size() < 8 || !marker(sf, 0, "KMCS") || !marker(sf, sf.size() - 4, "KMCS")) {
    ctx_set_error(ctx, "database markers missing");
    return KMC_ERR_INVALID_ARG;
  }
  const uint32_t hlen = get32(pf.data() + pf.size() - 8);
  if (hlen < 68 || (uint64_t)hlen + 12 > pf.size()) {
    ctx_set_error(ctx, "database header position out of range");
    return KMC_ERR_INVALID_ARG;
  }
  const uint8_t* h = pf.data() + pf.size() - 8 - hlen;
  kmc_db* db = new (std::nothrow) kmc_db();
  if (!db) return KMC_ERR_OUT_OF_MEMORY;
  db->device = ctx_device(ctx);
  kmc_db_info& I = db->info;
  I.kmer_length = get32(h);
  I.mode = get32(h + 4);
  I.counter_size = get32(h + 8);
  I.lut_prefix_length = get32(h + 12);
  I.signature_length = get32(h + 16);
  I.min_count = get32(h + 20);
  I.max_count = get32(h + 24);
  I.total_kmers = get64(h + 28);
  I.flags = get32(h + 36) & (KMC_FLAG_NON_CANONICAL | KMC_FLAG_PLAIN_MINIMIZERS);
  const uint64_t L = I.lut_prefix_length <= 14 ? 1ull << (2 * I.lut_prefix_length) : 0;
  const uint64_t n_sig =
      I.signature_length <= 12 ? (1ull << (2 * I.signature_length)) + 1 : 0;
  // prefixes + map fill the space between the marker and the header
  const uint64_t between = pf.size() - 8 - hlen - 4;
  if (I.mode != 0 || !L || !n_sig || between < n_sig * 4 || (between - n_sig * 4) % 8 != 0 ||
      (between - n_sig * 4) / 8 < 1 || ((between - n_sig * 4) / 8 - 1) % L != 0) {
    ctx_set_error(ctx, "database sizes do not match its header");
    delete db;
    return KMC_ERR_INVALID_ARG;
  }
  const uint64_t n_pre = (between - n_sig * 4) / 8;
  db->n_bins = (uint32_t)((n_pre - 1) / L);
  std::string why;
  if (!shape(db, why) ||
      sf.size() != 8 + I.total_kmers * (uint64_t)db->rec_bytes) {
    ctx_set_error(ctx, why.empty() ? "suffix file size does not match the header" : why.c_str());
    delete db;
    return KMC_ERR_INVALID_ARG;
  }
  std::vector<uint64_t> pre(n_pre);
  for (uint64_t i = 0; i < n_pre; ++i) pre[i] = get64(pf.data() + 4 + 8 * i);
  std::vector<uint32_t> map(n_sig);
  for (uint64_t i = 0; i < n_sig; ++i) {
    map[i] = get32(pf.data() + 4 + 8 * n_pre + 4 * i);
    if (map[i] >= db->n_bins) {
      ctx_set_error(ctx, "database map entry beyond its prefix arrays");
      delete db;
      return KMC_ERR_INVALID_ARG;
    }
  }
  if (pre[0] != 0 || pre[n_pre - 1] != I.total_kmers) {
    ctx_set_error(ctx, "database prefix arrays do not span the records");
    delete db;
    return KMC_ERR_INVALID_ARG;
  }
  for (uint64_t i = 1; i < n_pre; ++i) {
    if (pre[i] < pre[i - 1]) {
      ctx_set_error(ctx, "database prefix arrays are not ascending");
      delete db;
      return KMC_ERR_INVALID_ARG;
    }
  }
  if (hipSetDevice(db->device) != hipSuccess) {
    (void)hipGetLastError();
    delete db;
    return KMC_ERR_DEVICE;
  }
  const uint64_t nrec = I.total_kmers * db->rec_bytes;
  if (!dev_alloc(&db->map, n_sig) || !dev_alloc(&db->pre, n_pre) || !dev_alloc(&db->rec, nrec + kRecPad)) {
    free_parts(db);
    return KMC_ERR_OUT_OF_MEMORY;
  }
  if (hipMemcpy(db->map, map.data(), n_sig * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(db->pre, pre.data(), n_pre * 8, hipMemcpyHostToDevice) != hipSuccess ||
      (nrec && hipMemcpy(db->rec, sf.data() + 4, nrec, hipMemcpyHostToDevice) != hipSuccess)) {
    (void)hipGetLastError();
    free_parts(db);
    return KMC_ERR_DEVICE;
  }
  *out = db;
  return KMC_OK;
}

kmc_status kmc_db_query(const kmc_db* db, const uint64_t* kmers, uint64_t n, uint32_t min_count,
                        uint32_t max_count, uint32_t* counts, void* stream) {
  if (!db || (n && (!kmers || !counts))) return KMC_ERR_INVALID_ARG;
  if (n == 0) return KMC_OK;
  if (hipSetDevice(db->device) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DbView D = view(db);
  if (db->info.kmer_length <= 32)
    hipLaunchKernelGGL(k_db_query<1>, dim3(grid(n)), dim3(256), 0, s, D, kmers, n, min_count,
                       max_count, counts);
  else
    hipLaunchKernelGGL(k_db_query<2>, dim3(grid(n)), dim3(256), 0, s, D, kmers, n, min_count,
                       max_count, counts);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  return KMC_OK;
}

kmc_status kmc_db_decode(const kmc_db* db, uint64_t* keys, uint32_t* counts, void* stream) {
  if (!db || (db->info.total_kmers && (!keys || !counts))) return KMC_ERR_INVALID_ARG;
  const uint64_t n = db->info.total_kmers;
  if (n == 0) return KMC_OK;
  if (hipSetDevice(db->device) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DbView D = view(db);
  const uint64_t n_slots = (uint64_t)db->n_bins << (2 * db->info.lut_prefix_length);
  if (db->info.kmer_length <= 32)
    hipLaunchKernelGGL(k_db_decode<1>, dim3(grid(n)), dim3(256), 0, s, D, n_slots, n, keys,
                       counts);
  else
    hipLaunchKernelGGL(k_db_decode<2>, dim3(grid(n)), dim3(256), 0, s, D, n_slots, n, keys,
                       counts);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  return KMC_OK;
}

void kmc_db_free(kmc_db* db) { free_parts(db); }

}  // extern "C"
