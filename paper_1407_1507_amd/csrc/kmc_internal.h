// Internal declarations shared by the kernels and the host runtime of
// libkmc_hip.so.  Not part of the public ABI (include/kmc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kmc.h"

namespace kmc {

// Sizes of the work units.
constexpr int kExpandThreads = 256;      // threads of the expansion kernels: records per round
// Records per expansion task, by key width (a multiple of kExpandThreads):
// more records per task give longer runs of keys per (task, tile), so fewer
// partially written lines.
constexpr uint32_t kExpandTask1 = 256;
constexpr uint32_t kExpandTask2 = 256;
inline uint32_t expand_task_records(uint32_t key_words) {
  return key_words == 1 ? kExpandTask1 : kExpandTask2;
}
constexpr int kSortThreads = 256;        // threads of a tile-sort workgroup
constexpr int kTileCap1 = 4096;          // keys of one LDS tile (1-word keys)
constexpr int kTileCap2 = 2048;          // same, 2-word keys
constexpr int kMaxFineBits = 12;         // fine ranges per bin: at most 2^12
constexpr int kMaxTilesPerBin = 1 << kMaxFineBits;  // a tile holds >= 1 fine range
// Most super k-mer records one bin's region may hold: the lane scan addresses a
// workgroup's slots in a bin by 32-bit offsets (kMaxBinRecords plus a
// workgroup's slot count stays below 2^31).
constexpr uint64_t kMaxBinRecords = (1ull << 31) - (1ull << 20);

// Parameters of the split (signature scan) kernels.
struct ScanCfg {
  uint32_t k, p, w;      // w = k - p + 1: most k-mers in one super k-mer
  uint32_t filter;       // 1: signatures (AAA/ACA/AA filter), 0: plain minimizers
  uint32_t pmask;        // 2p low bits
  uint32_t sent;         // 4^p: signature of a k-mer with no allowed p-mer
  uint32_t n_bins;
  uint32_t seq_align;    // alignment of seq (16, 4 or 1): widest loads it allows
  uint32_t L;            // floor(log2 w): the wide scan joins two 2^L windows
};

// One expansion task: records [rec_begin, rec_end) of bin `bin`.
struct ExpandTask {
  uint64_t rec_begin;
  uint32_t n_rec;
  uint32_t bin;
};

// Tasks of a per-record kernel: bin b's records [rec_base[b], rec_end[b]) in
// runs of `per`, tasks pre[b] .. pre[b+1] - 1; bin[t] is the bin of task t
// (filled on the device by launch_task_bins), or, when desc is set, desc[t]
// is task t whole (one load instead of two dependent ones).
struct TaskMap {
  const uint16_t* bin;
  const uint64_t* pre;
  const uint64_t* rec_base;
  const uint64_t* rec_end;
  uint32_t per;
  const ExpandTask* desc;
  __device__ __forceinline__ ExpandTask get(uint32_t t) const {
    if (desc) return desc[t];
    ExpandTask k;
    k.bin = bin[t];
    k.rec_begin = rec_base[k.bin] + (uint64_t)(t - pre[k.bin]) * per;
    const uint64_t left = rec_end[k.bin] - k.rec_begin;
    k.n_rec = left < per ? (uint32_t)left : per;
    return k;
  }
};

// One sort tile: keys [begin, begin + size) of the key buffer.
struct Tile {
  uint64_t begin;
  uint32_t size;
  uint32_t bin;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return the launch status.

// Signature histograms of reads r with r % stride == 0: hist[sig] = k-mers,
// hist[4^p + 1 + sig] = super k-mers; sample[0] += k-mers, sample[1] += bases.
hipError_t launch_sig_hist(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                           uint64_t n_reads, uint64_t n_bases, uint64_t stride,
                           const ScanCfg& cfg, uint32_t key_words, uint32_t* hist,
                           unsigned long long* sample);

// Write every super k-mer record into its bin's region [cap_base[b],
// cap_base[b+1]).  cursor[b] starts at cap_base[b] and counts every record of
// bin b (records past the region end are counted but not written);
// kmer_cnt[b] += k-mers of bin b.
hipError_t launch_split_scatter(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                                uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                                uint32_t key_words, const uint32_t* sig_to_bin,
                                unsigned long long* cursor, unsigned long long* kmer_cnt,
                                const uint64_t* cap_base, uint64_t* records);

// Per-window signature and super k-mer starts (audit).
// The split and the debug scan with one position per lane (kmc_scan_wide.hip),
// for windows whose per-lane buffers do not fit LDS well.
hipError_t launch_split_wide(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                             uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                             uint32_t key_words,
                             const uint32_t* sig_to_bin, unsigned long long* cursor,
                             unsigned long long* kmer_cnt, const uint64_t* cap_base,
                             uint64_t* records);
// Signature histogram of every stride-th read with the position-per-lane
// scan (one read per wavefront when stride > 1): for long reads.
hipError_t launch_sig_hist_wide(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                                uint64_t n_reads, uint64_t stride, const ScanCfg& cfg,
                                uint32_t key_words, uint32_t* hist, unsigned long long* sample);
hipError_t launch_debug_wide(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                             uint64_t n_reads, const ScanCfg& cfg, uint32_t key_words,
                             uint32_t* sig, uint8_t* start);

hipError_t launch_debug_sigs(hipStream_t s, const uint8_t* seq, const uint64_t* offsets,
                             uint64_t n_reads, uint64_t n_bases, const ScanCfg& cfg,
                             uint32_t key_words, uint32_t* sig, uint8_t* start);

// Parameters of the expansion / sort kernels.
struct KeyCfg {
  uint32_t k;
  uint32_t key_words;
  uint32_t fine_bits;   // fine ranges per bin = 2^fine_bits (top bits of the key)
  uint32_t tile_limit;  // tiles are packed up to this many keys
  uint32_t tile_cap;    // keys one LDS tile can hold
  uint32_t n_bins;
  uint32_t cutoff_min, cutoff_max;
  uint32_t fp_bits;     // fingerprint bits of 128-bit hash-table claims (47; fewer in tests)
  uint32_t canonical;   // 1: keys are canonical k-mers; 0: forward k-mers as read
  uint32_t counter_max; // stored counts saturate here (0xFFFFFFFF: exact)
  // (k,x)-mers: x (0: off) and the pass: 1 = the (k,x)-mers of the records
  // are the keys (64-bit: x' in the top two bits, the canonical (k + x')-mer
  // left-aligned below); 2 = the records are distinct (k,x)-mers with their
  // counts (word 0 the key, word 1 count << 8 | k-mers) and the keys are
  // their k-mers, each weighted by the (k,x)-mer's count
  uint32_t kx = 0;
  uint32_t kx_pass = 0;
  // a tile over tile_limit (a big tile) also takes the fine ranges after it
  // while it holds at most big_merge keys (0: a big tile is one range)
  uint32_t big_merge = 0;
};

// bin[t] for every task t of two task maps (pre arrays of n_bins + 1).
hipError_t launch_task_bins(hipStream_t s, uint32_t n_bins, const uint64_t* pre_a,
                            uint16_t* bin_a, const uint64_t* pre_b, const uint64_t* rec_base,
                            const uint64_t* rec_end, uint32_t per_b, ExpandTask* desc_b);

// Fine-range histogram of every bin: fine_hist[bin << fine_bits | range].
hipError_t launch_fine_hist(hipStream_t s, const KeyCfg& kc, const TaskMap& tm,
                            uint32_t n_tasks, const uint64_t* records, uint32_t* fine_hist);

// Per bin: fine ranges -> tiles.  Writes tile_of_fine (local tile id per
// range), tiles[tile_base[b] + t] and fills cursors with each tile's start.
hipError_t launch_plan_tiles(hipStream_t s, const KeyCfg& kc, const uint32_t* fine_hist,
                             const uint64_t* key_base, const uint64_t* tile_base,
                             uint16_t* tile_of_fine, Tile* tiles,
                             unsigned long long* tile_cursor);

// Expand every record into canonical keys and scatter them into their tiles.
// Tasks hold at most expand_task_records(key_words) records.
hipError_t launch_expand_scatter(hipStream_t s, const KeyCfg& kc, const TaskMap& tm,
                                 uint32_t n_tasks, const uint64_t* records,
                                 const uint16_t* tile_of_fine, const uint64_t* tile_base,
                                 const uint64_t* key_base, uint32_t max_tiles_per_bin,
                                 unsigned long long* tile_cursor, uint64_t* keys,
                                 uint32_t* weights = nullptr);

// (k,x)-mers, between the two passes: the distinct (k,x)-mers of the first
// pass (keys, counts; n of them) as records of the second, two words each:
// the key, then count << 8 | the number of its k-mers.
hipError_t launch_kx_records(hipStream_t s, const uint64_t* keys, const uint32_t* counts,
                             uint64_t n, uint64_t* records);

// Sort + count every tile that fits LDS.  Output of a tile is written over
// its own keys (out_counts at the same indices); tile_out[t] = entries kept,
// tile_distinct[t] = distinct keys of tile t.  Tiles larger than LDS are appended to
// big_list (count in n_big[0]) with their size in big_size and a private
// slice of the HBM scratch at big_off (its size summed into big_total).
// weighted (64-bit keys only): out_counts[i] holds the weight of key i on
// entry, each key standing for that many equal keys.
hipError_t launch_tile_sort(hipStream_t s, const KeyCfg& kc, const Tile* tiles,
                            uint64_t n_tiles, uint64_t* keys, uint32_t* out_counts,
                            uint32_t* tile_out, uint32_t* big_list, uint64_t* big_off,
                            uint32_t* n_big, unsigned long long* big_total,
                            uint32_t* tile_distinct, uint32_t* big_size, bool weighted);

// Sort + count the big tiles: MSD partition through HBM, each tile
// ping-ponging between its keys and its own slice tmp[big_off[i] ...]; for
// 64-bit keys each big tile is first streamed through the LDS hash table and
// partitioned only if it has too many distinct keys; with stream_first that
// pass is a kernel of its own (more workgroups per compute unit) that lists
// the failures in fail_list for the partition kernel.  The number of big tiles is read on the device (*n_big, final
// once the tile kernel has run); workgroups take tiles from the counters
// *next and *fail_next, and the failures are counted in *n_fail (all three
// zero at launch).  order and fail_list hold max_big entries; max_big bounds
// *n_big (the grids never exceed it).  *big_out accumulates the entries the
// big tiles keep.  tmpw (64-bit keys, weighted tiles): u32 scratch beside
// tmp for the weights, which move with their keys; null when unweighted.
hipError_t launch_big_tiles(hipStream_t s, const KeyCfg& kc, const Tile* tiles,
                            const uint32_t* big_list, const uint64_t* big_off,
                            const uint32_t* big_size, uint32_t* order,
                            uint32_t* fail_list, const uint32_t* n_big, uint32_t* next,
                            uint32_t* n_fail, uint32_t* fail_next, uint64_t max_big,
                            bool stream_first,
                            uint64_t* keys, uint64_t* tmp, uint32_t* out_counts, uint32_t* tmpw,
                            uint32_t* tile_out, uint32_t* tile_distinct,
                            unsigned long long* big_out);

// Exclusive scan of n uint32 into uint64 (out has n + 1 entries: out[n] = total).
hipError_t launch_scan_u32(hipStream_t s, const uint32_t* in, uint64_t n, uint64_t* out,
                           uint64_t* block_tmp);
uint64_t scan_tmp_words(uint64_t n);

// Copy every tile's kept entries to out_keys/out_counts at tile_off[t].
hipError_t launch_gather(hipStream_t s, const KeyCfg& kc, const Tile* tiles, uint64_t n_tiles,
                         const uint64_t* tile_off, const uint64_t* keys,
                         const uint32_t* counts, uint64_t* out_keys, uint32_t* out_counts);

// Global ascending order of the kept entries (instead of bin-major): entries
// are partitioned by their top seg_bits key bits into segments, segments are
// packed into groups starting at the first segment at or above each multiple
// of `group` entries, and each group is put in order.
struct AscPlan {
  uint32_t seg_bits;  // segments: 2^seg_bits (at most kMaxSegBits)
  uint64_t group;     // group stride in entries (CAP / 2 of the key width)
  uint64_t n_groups;  // ceil(n_out / group)
};
constexpr uint32_t kMaxSegBits = 20;
// Plan for n_out entries of keys of 2k bits.
AscPlan plan_ascending(uint64_t n_out, uint32_t k, uint32_t key_words);
// The bin-major table (table_keys / table_counts, n_out entries) put in
// ascending order in place.  seg_cnt: u32[2^seg_bits]; seg_start:
// u64[2^seg_bits + 1]; scan_tmp: scan_tmp_words(2^seg_bits); lo:
// u64[n_groups + 1]; xk / xc: scratch of n_out entries (not aliasing the
// table).
hipError_t launch_ascending(hipStream_t s, const KeyCfg& kc, uint64_t n_out, const AscPlan& ap,
                            uint32_t* seg_cnt, uint64_t* seg_start, uint64_t* scan_tmp,
                            uint64_t* lo, uint64_t* xk, uint32_t* xc, uint64_t* table_keys,
                            uint32_t* table_counts);

// out[b] = tile_off[tile_base[b]] for b in [0, n_bins] (first output entry of each bin).
hipError_t launch_bin_offsets(hipStream_t s, const uint64_t* tile_off, const uint64_t* tile_base,
                              uint32_t n_bins, uint64_t* out);


// Validate a device offsets array: err[0] |= 1 if offsets[0] != 0, not
// non-decreasing, or offsets[n_reads] != n_bases.
hipError_t launch_check_offsets(hipStream_t s, const uint64_t* offsets, uint64_t n_reads,
                                uint64_t n_bases, uint32_t* err);

}  // namespace kmc

struct kmc_ctx;
namespace kmc {
// Extension slot of a context: *slot holds an object released by `release`
// (registered on first use) when the context is destroyed.
void** ctx_ext(kmc_ctx* c, void (*release)(void*));
int ctx_device(const kmc_ctx* c);
hipStream_t ctx_stream(const kmc_ctx* c);
void ctx_set_error(kmc_ctx* c, const char* msg);
// Free the context's cached device buffers (after a one-off large job).
void ctx_release_buffers(kmc_ctx* c);
// Device buffer `slot` of the context's cache (grown to `bytes` as needed and
// kept for later calls; freed with the context), or nullptr on failure.
constexpr int kCtxAuxBuffers = 12;
void* ctx_aux_buffer(kmc_ctx* c, int slot, size_t bytes);
// Set the context's memory budget (as kmc_ctx_set_budget).
void ctx_set_budget(kmc_ctx* c, uint64_t bytes);
// Lend the context a device region: its buffers are released, and until
// ctx_end_region every device buffer of its jobs is taken from the region
// (a job that needs more fails with KMC_ERR_OUT_OF_MEMORY).  Pair it with a
// budget no larger than the region.
void ctx_lend_region(kmc_ctx* c, void* base, size_t bytes);
// Give the region back (after the stream is idle); the context allocates its
// own buffers again.
void ctx_end_region(kmc_ctx* c);
// Knobs: copy src's override and tuned knobs into dst; tuned knobs of the
// class of (key_words, n_bases); the batch pool's worker count (0 = default);
// override (k non-null) or clear it, returning whether one was set.
void ctx_copy_tuning(kmc_ctx* dst, const kmc_ctx* src);
void ctx_set_tuned(kmc_ctx* c, uint32_t key_words, uint64_t n_bases, const kmc_knobs& k);
uint32_t ctx_batch_workers(const kmc_ctx* c);
void ctx_set_batch_workers(kmc_ctx* c, uint32_t n);
bool ctx_override_knobs(kmc_ctx* c, const kmc_knobs* k);
// kmc_count_ws; with own_table a device table is allocated apart from the
// workspace, so it outlives the workspace's reuse.
kmc_status count_ws_impl(kmc_ctx* c, const kmc_reads* reads, const kmc_params* params,
                         void* stream, void* workspace, size_t ws_bytes, bool own_table,
                         kmc_table** out);
// kmc_count_static with `scratch` (scratch_bytes, 256-byte aligned device
// memory) as the workspace and the table written to keys_out / counts_out.
kmc_status count_static_impl(kmc_ctx* c, const kmc_reads* reads, const kmc_params* params,
                             void* stream, void* scratch, size_t scratch_bytes,
                             uint64_t* keys_out, uint32_t* counts_out, uint64_t out_cap,
                             uint64_t* n_out, uint64_t* bin_offsets, kmc_stats* stats);
}  // namespace kmc
