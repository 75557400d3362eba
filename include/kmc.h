/*
 * kmc.h -- C ABI of the MI355X k-mer counting library (libkmc_hip.so).
 *
 * The library computes, for a set of DNA reads, every canonical k-mer with its
 * exact number of occurrences, following the method of KMC 2 (Deorowicz,
 * Kokot, Grabowski, Debudaj-Grabysz, 2014):
 *   1. each read is split into super k-mers: maximal runs of consecutive
 *      k-mers that share one signature (Methods, "From minimizers to
 *      signatures" and "Sketch of the algorithm", Fig. 1);
 *   2. the 4^p signatures are merged into n_bins bins from a histogram of a
 *      small sample of the input (Methods, "Sketch of the algorithm"), and
 *      every super k-mer is sent to the bin of its signature;
 *   3. each bin is expanded into canonical k-mers (the smaller of a k-mer and
 *      its reverse complement, Methods, "Minimizers of k-mers"), radix sorted
 *      and run-length counted; k-mers counted fewer than cutoff_min or more
 *      than cutoff_max times are dropped (Methods, "Additional features";
 *      supplement, -ci / -cx).
 * Every step runs in hand-written HIP kernels on the GPU; bins live in HBM.
 *
 * Symbols: A=0 C=1 G=2 T=3 (either case); a k-mer key packs its symbols with
 * the leftmost symbol in the most significant bits (supplement, database
 * format), so numeric order is lexicographic order.  Any other byte (N, IUPAC
 * codes, ...) is invalid: every window holding one is skipped.
 *
 * Conventions for every call:
 *   - Nothing throws across this ABI; every call returns a kmc_status.
 *   - On error *out is set to NULL and nothing is leaked; no partial table.
 *   - Inputs are borrowed for the duration of the call only.
 *   - One kmc_ctx must not be used by two host threads at the same time.
 */
#ifndef KMC_H_
#define KMC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kmc_status {
  KMC_OK = 0,
  KMC_ERR_INVALID_ARG = 1,   /* an argument failed validation (see kmc_count) */
  KMC_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
  KMC_ERR_DEVICE = 3,        /* a HIP call failed; text via kmc_last_error */
  KMC_ERR_TOO_LARGE = 4,     /* the job exceeds a size limit of the library */
  KMC_ERR_BUSY = 5           /* reserved for asynchronous forms */
} kmc_status;

/* Reads in CSR form.  seq holds n_bases bytes (ASCII); read i is
 * seq[offsets[i] .. offsets[i+1]).  offsets has n_reads + 1 entries,
 * offsets[0] == 0, non-decreasing, offsets[n_reads] == n_bases.
 * on_device = 0: both arrays are host memory; 1: both are device memory of
 * the context's device (e.g. torch tensors on cuda:0). */
typedef struct kmc_reads {
  const uint8_t* seq;
  const uint64_t* offsets;
  uint64_t n_reads;
  uint64_t n_bases;
  int32_t on_device;
  int32_t reserved;
} kmc_reads;

/* Counting parameters.
 *   k           k-mer length, 4 <= k <= 64 (keys are 1 word for k <= 32,
 *               2 words for k > 32);
 *   p           signature length, 4 <= p <= min(k, 12);
 *   n_bins      number of bins, 1 <= n_bins <= min(4^p + 1, 65535);
 *   cutoff_min  keep a k-mer only if its count >= cutoff_min (0 acts as 1);
 *   cutoff_max  keep a k-mer only if its count <= cutoff_max;
 *               cutoff_min <= cutoff_max;
 *   flags       KMC_FLAG_* bits;
 *   counter_max stored counts saturate at this value (0 = exact counts);
 *               the cutoffs apply to the exact counts (supplement, -cs:
 *               the maximal value of a counter). */
typedef struct kmc_params {
  uint32_t k;
  uint32_t p;
  uint32_t n_bins;
  uint32_t cutoff_min;
  uint32_t cutoff_max;
  uint32_t flags;
  uint32_t counter_max;
} kmc_params;

/* The returned table stays in device memory (kmc_table.on_device = 1) instead
 * of being copied to host memory. */
#define KMC_FLAG_DEVICE_TABLE 0x1u
/* Plain canonical minimizers instead of signatures (no AAA/ACA/AA filter;
 * Methods, "Minimizers of k-mers").  Changes only the bins, never the counts. */
#define KMC_FLAG_PLAIN_MINIMIZERS 0x2u
/* Entries in ascending key order over the whole table instead of grouped by
 * bin (then kmc_table.bin_offsets is NULL).  Same entries either way. */
#define KMC_FLAG_ASCENDING 0x4u
/* Count k-mers as read instead of in canonical form (supplement, -b: turn
 * off the canonical form): a k-mer and its reverse complement are counted
 * as two keys.  Bins are unchanged (the signature of a k-mer and of its
 * reverse complement are the same). */
#define KMC_FLAG_NON_CANONICAL 0x8u
/* (k,x)-mers (Methods, "(k,x)-mers" and the counting from sorted (k,x)-mers
 * that follows Fig. 2): each super k-mer is cut into the fewest (k + x')-mers,
 * x' <= x, whose k-mers are all canonical in the same direction (a piece grows
 * while the next k-mer has the direction of its first and it holds at most
 * x + 1 k-mers; a k-mer is forward when it is not larger than its reverse
 * complement), each stored in the direction that makes its k-mers canonical.
 * These are sorted and run-length counted per bin, and the k-mer counts are
 * taken from the distinct (k,x)-mers, each of whose k-mers counts as many
 * times as the (k,x)-mer occurs.  The table is the same as without the flag.
 * x = 1..3 in bits 4-5 (KMC_FLAG_KX(x)); needs canonical k-mers and
 * k + x <= 31; not available with a caller workspace (kmc_count_ws,
 * kmc_count_static) or a memory budget that splits the job into bin groups
 * (KMC_ERR_INVALID_ARG). */
#define KMC_FLAG_KX(x) (((uint32_t)(x) & 3u) << 4)
#define KMC_FLAG_KX_MASK 0x30u
/* Test only.  Tiles of 128-bit keys (k > 32) are counted in an LDS hash table
 * whose slots are claimed by a 47-bit fingerprint of the key; a tile where two
 * different keys share a fingerprint is detected and counted by the exact
 * partition path for tiles too large for LDS instead.  This flag narrows the
 * fingerprint to 2 bits, so almost every tile with several distinct keys takes
 * that path: the table is the same, and tests use the flag to drive it. */
#define KMC_FLAG_TEST_NARROW_FINGERPRINT 0x100u

/* Kernels timed in kmc_stats.us_kernel. */
enum {
  KMC_K_SIG_HIST = 0,   /* signature histogram of the sample */
  KMC_K_SPLIT = 1,      /* signature scan, super k-mers into bins */
  KMC_K_FINE_HIST = 2,  /* key histogram per bin (top bits) */
  KMC_K_PLAN_TILES = 3, /* fine ranges -> sort tiles */
  KMC_K_EXPAND = 4,     /* canonical keys into tiles */
  KMC_K_TILE_SORT = 5,  /* LDS sort, run-length count, cutoffs */
  KMC_K_BIG_TILES = 6,  /* tiles larger than LDS */
  KMC_K_ASSEMBLE = 7,   /* scan of tile outputs and gather */
  KMC_N_KERNELS = 8
};

/* Per-job statistics (measured on the device). */
typedef struct kmc_stats {
  uint64_t n_reads;
  uint64_t n_bases;
  uint64_t n_kmers;        /* valid windows = sum of counts before cutoffs */
  uint64_t n_superkmers;   /* records written to the bins */
  uint64_t n_distinct;     /* distinct canonical k-mers before cutoffs */
  uint64_t n_out;          /* entries kept after cutoffs */
  uint64_t sample_kmers;   /* k-mers in the signature histogram sample */
  uint64_t max_bin_kmers;  /* k-mers in the largest bin */
  uint64_t n_tiles;        /* sort tiles (sub-bins held in LDS) */
  uint64_t n_big_tiles;    /* tiles too large for LDS, sorted in HBM */
  uint64_t bytes_alg;      /* algorithmic HBM bytes of the job */
  uint64_t split_passes;   /* 1, or 2 when a bin outgrew its sampled estimate */
  uint64_t n_big_keys;     /* k-mers of the tiles counted through HBM (n_big_tiles) */
  uint64_t n_big_out;      /* entries of the table those tiles kept */
  uint64_t n_groups;       /* bin groups of the sorting phase (1 unless a
                              memory budget splits the job) */
  uint64_t records_spilled; /* 1 if the super k-mer records went to pinned
                               host memory (memory budget) */
  uint64_t n_kx_entries;   /* KMC_FLAG_KX: (k,x)-mers sorted (Table 7's sorted
                              fraction is n_kx_entries / n_kmers); else 0 */
  uint64_t n_kx_distinct;  /* KMC_FLAG_KX: distinct (k,x)-mers; else 0 */
  double us_map;           /* device time of each phase, microseconds */
  double us_split;
  double us_expand;
  double us_sort;
  double us_assemble;
  double us_total;         /* first kernel to last kernel */
  double us_kernel[8];     /* device time of each kernel (KMC_K_*), microseconds */
  double us_queue;         /* served jobs: submit -> start of work, microseconds */
  double us_latency;       /* served jobs: submit -> table ready, microseconds */
} kmc_stats;

/* Result of a count.  Entries are grouped by bin (bin b holds entries
 * [bin_offsets[b], bin_offsets[b+1])), the order of the paper's database
 * (signature, then k-mer; supplement, database format), and ascending by key
 * inside each bin.  Bins hold disjoint key sets.  With KMC_FLAG_ASCENDING the
 * entries are in ascending key order over the whole table and bin_offsets is
 * NULL.
 *   keys        n * key_words uint64; for key_words == 2 each key is stored
 *               hi word first, then lo word; the hi word holds the top
 *               2k - 64 bits;
 *   counts      n exact uint32 counts (no saturation);
 *   bin_offsets n_bins + 1 uint64 (always host memory; NULL in ascending
 *               order);
 *   sig_to_bin  4^p + 1 uint32: bin of every signature value; the last entry
 *               is for k-mers with no allowed p-mer (always host memory).
 * keys/counts are host memory unless on_device = 1.  reserved records how
 * the library owns keys/counts (1: in a caller's workspace, kmc_count_ws;
 * 2: a device block, 3: a pinned host block, that kmc_table_free hands back
 * to the library's pool of table memory for later tables); callers leave it
 * alone.
 * The table is owned by the library: release it with kmc_table_free. */
typedef struct kmc_table {
  uint32_t k;
  uint32_t key_words;
  uint64_t n;
  uint64_t* keys;
  uint32_t* counts;
  uint32_t n_bins;
  uint32_t p;
  uint64_t* bin_offsets;
  uint32_t* sig_to_bin;
  int32_t on_device;
  int32_t reserved;
  kmc_stats stats;
} kmc_table;

typedef struct kmc_ctx kmc_ctx;

/* Create a context on HIP device `device` (its workspace, cached between
 * calls, and its default stream).  Returns KMC_ERR_DEVICE if the device is
 * not usable. */
kmc_status kmc_ctx_create(int device, kmc_ctx** out);
/* Destroy a context and free its workspace.  NULL is allowed. */
void kmc_ctx_destroy(kmc_ctx* ctx);
/* Text of the last error seen on ctx ("" if none).  Valid until the next
 * call on ctx. */
const char* kmc_last_error(const kmc_ctx* ctx);
/* Memory budget of ctx's jobs (kmc_count / kmc_count_ex): the device bytes
 * their buffers may take (the caller's reads and the returned device table
 * aside); 0 = no bound (the default).  A job above it still runs, the way
 * the paper's disk-based design keeps RAM bounded (bins on disk, one bin
 * group sorted at a time; Methods, "Sketch of the algorithm"; Additional
 * features, RAM-only mode): its bins are expanded, counted and assembled in
 * groups whose keys fit the budget, and when the super k-mer records take
 * more than half of it they go to pinned host memory and each group's
 * records are copied back to the device.  Same table.  KMC_ERR_TOO_LARGE if
 * one bin's keys exceed the budget.  With KMC_FLAG_ASCENDING the whole table
 * is ordered on the device.  Not used by kmc_count_ws / kmc_count_static
 * (their workspace is the bound). */
kmc_status kmc_ctx_set_budget(kmc_ctx* ctx, uint64_t device_bytes);

/* Knobs of the counting path.  None changes the table (entries, counts,
 * bins and order); they trade work between kernels:
 *   tile_fill       sort tiles are packed up to tile_fill quarters of the
 *                   LDS tile (2 or 3; 0 = 3);
 *   fine_bits_bias  added to the number of key bits (fine ranges per bin)
 *                   the plan picks for the first digit, -2..2 (then clamped
 *                   to 1..12);
 *   expand_task     super k-mer records per expansion task: 256, 512 or
 *                   1024 (0 = the default for the key width).
 * Jobs counted in a caller's workspace (kmc_count_ws, kmc_count_static, the
 * served form) use the defaults. */
typedef struct kmc_knobs {
  uint32_t tile_fill;
  int32_t fine_bits_bias;
  uint32_t expand_task;
} kmc_knobs;

/* Knobs for every later job of ctx (NULL: back to the defaults, or to the
 * knobs kmc_autotune chose).  KMC_ERR_INVALID_ARG for a value out of range. */
kmc_status kmc_ctx_set_knobs(kmc_ctx* ctx, const kmc_knobs* knobs);

/* Count the canonical k-mers of `reads` (see the header comment).
 * Uses a context on device 0 owned by the calling host thread.
 * Validation (KMC_ERR_INVALID_ARG): see kmc_params; reads != NULL, out !=
 * NULL, seq/offsets non-NULL when n_reads > 0, offsets well formed.
 * Reads shorter than k and empty inputs contribute nothing; an empty table
 * (n = 0) is a valid result. */
kmc_status kmc_count(const kmc_reads* reads, uint32_t k, uint32_t p, uint32_t n_bins,
                     uint32_t cutoff_min, uint32_t cutoff_max, kmc_table** out);

/* As kmc_count, on context ctx, with explicit parameters, on HIP stream
 * `stream` (a hipStream_t; NULL = the context's stream).  The call returns
 * when the table is complete. */
kmc_status kmc_count_ex(kmc_ctx* ctx, const kmc_reads* reads, const kmc_params* params,
                        void* stream, kmc_table** out);

/* Free a table returned by this library.  NULL is allowed. */
void kmc_table_free(kmc_table* table);

/* Static text for a status code. */
const char* kmc_status_str(kmc_status status);

/* One counting job: reads + parameters.  The reads are borrowed until the
 * job's table has been returned. */
typedef struct kmc_job {
  kmc_reads reads;
  kmc_params params;
} kmc_job;

/* Device bytes that kmc_count_ws may use for this job, computed from the sizes
 * alone (an upper bound: every window a k-mer, every bin at its largest).
 * Returns KMC_ERR_INVALID_ARG under the same rules as kmc_count. */
kmc_status kmc_workspace_size(const kmc_reads* reads, const kmc_params* params, size_t* bytes);

/* As kmc_count_ex, with every device buffer of the job carved from
 * `workspace` (device memory of ctx's device, at least kmc_workspace_size
 * bytes, 256-byte aligned); the library allocates no device memory of its
 * own for the job.  With KMC_FLAG_DEVICE_TABLE the table's keys/counts also
 * live in the workspace: they stay valid until the workspace is reused, and
 * kmc_table_free releases only the host parts.  Returns KMC_ERR_OUT_OF_MEMORY
 * if ws_bytes is too small. */
kmc_status kmc_count_ws(kmc_ctx* ctx, const kmc_reads* reads, const kmc_params* params,
                        void* stream, void* workspace, size_t ws_bytes, kmc_table** out);

/* Count n_jobs independent jobs (uneven sizes and parameters allowed).
 * Jobs run concurrently on a pool of worker streams owned by ctx, each with
 * its own workspace; outs[i] receives job i's table, identical to what
 * kmc_count_ex returns for that job alone.  On any failure every outs[i] is
 * NULL, nothing is leaked, and the first failing job's status is returned. */
kmc_status kmc_batch_count(kmc_ctx* ctx, const kmc_job* jobs, uint32_t n_jobs, kmc_table** outs);

/* Autotuner.  For each class of the given jobs (key width, and the power of
 * two of its input bases) the largest job of the class is counted alone with
 * every candidate knob set (kmc_knobs: tile packing 2/4 or 3/4, first-digit
 * bits -1..+1, 256 / 512 / 1024 records per expansion task; twelve sets),
 * and the fastest device time is kept as the class's knobs for later jobs of
 * ctx (kmc_count_ex and kmc_batch_count; a kmc_ctx_set_knobs override
 * wins).  Then up to 64 of the jobs (spread over the list) run as one batch
 * with 2, 4 and 8 worker streams, and the fastest count becomes ctx's batch
 * pool size.  No knob
 * changes a table.  report may be NULL. */
#define KMC_TUNE_MAX_CLASSES 32
typedef struct kmc_tune_class {
  uint32_t key_words;
  uint32_t reserved;
  uint64_t sample_bases;
  kmc_knobs knobs;
  uint32_t pad;
  double us;           /* device time of the sample with the chosen knobs */
} kmc_tune_class;
typedef struct kmc_tune_report {
  uint32_t n_classes;
  uint32_t batch_workers;
  kmc_tune_class classes[KMC_TUNE_MAX_CLASSES];
} kmc_tune_report;
kmc_status kmc_autotune(kmc_ctx* ctx, const kmc_job* jobs, uint32_t n_jobs,
                        kmc_tune_report* report);

/* Served form: jobs are submitted while others run; a job is admitted when
 * its footprint (kmc_workspace_size) fits the HBM budget next to the jobs
 * already admitted, and up to max_active admitted jobs run at once, each on
 * its own stream; as one finishes the next admissible job starts (continuous
 * batching).  A job larger than the whole budget runs in a region of the
 * reserved arena: the whole arena less room for the largest other job queued
 * or running, when that leaves at least three quarters of it (that job runs
 * beside it), else the whole arena (the other jobs wait).  Its device
 * buffers are taken from that region and bounded by it as under
 * kmc_ctx_set_budget (bin groups, records in pinned host memory); its device
 * table, if requested, is allocated beside the budget. */
typedef struct kmc_server_cfg {
  uint64_t hbm_budget; /* bytes; 0 = 90% of the device memory free at start */
  uint32_t max_active; /* 1..16 jobs running at once; 0 = 4 */
  uint32_t reserved;
} kmc_server_cfg;

typedef struct kmc_server_stats {
  uint64_t submitted;
  uint64_t completed;
  uint64_t failed;
  uint64_t admitted_bytes;      /* footprint admitted now */
  uint64_t peak_admitted_bytes; /* largest admitted footprint so far */
  uint64_t budget;
  uint32_t active;              /* jobs running now */
  uint32_t queued;              /* jobs waiting for admission */
} kmc_server_stats;

typedef struct kmc_server kmc_server;

/* Start a server on ctx's device (ctx must outlive the server and must not
 * be used by the caller while the server runs). */
kmc_status kmc_server_start(kmc_ctx* ctx, const kmc_server_cfg* cfg, kmc_server** out);
/* Queue a job; *ticket identifies it.  The job's reads stay borrowed until
 * its table is polled. */
kmc_status kmc_server_submit(kmc_server* srv, const kmc_job* job, uint64_t* ticket);
/* Fetch a job's table: KMC_OK with *out set (the ticket is then released),
 * KMC_ERR_BUSY if it is not done and wait == 0, or the job's failure status.
 * wait != 0 blocks until the job is done.  stats.us_queue / us_latency give
 * the job's waiting time and its submit-to-ready latency. */
kmc_status kmc_server_poll(kmc_server* srv, uint64_t ticket, int32_t wait, kmc_table** out);
kmc_status kmc_server_stats_get(kmc_server* srv, kmc_server_stats* stats);
/* Stop accepting jobs, wait for running ones, free unpolled tables and the
 * server.  NULL is allowed. */
void kmc_server_stop(kmc_server* srv);

/* Allocation-free count, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same kernels as kmc_count_ws, with every scratch buffer
 * carved from a static device array of KMC_STATIC_SCRATCH_BYTES that each
 * device the library runs on holds from the first such call until the
 * process ends; the call makes no device or pinned-host allocation (host-side
 * planning uses ordinary heap memory).  The table is written to the caller's
 * device buffers, grouped by bin as in kmc_table (or in ascending key order
 * with KMC_FLAG_ASCENDING); KMC_FLAG_DEVICE_TABLE is implied.
 *   reads        host or device CSR reads (host reads are copied into the
 *                scratch first);
 *   stream       hipStream_t or NULL (the context's stream); the call returns
 *                when the table is complete;
 *   keys_out     device memory of ctx's device, out_cap * key_words uint64
 *                (key_words = 1 for k <= 32, else 2, hi word first);
 *   counts_out   device memory, out_cap uint32;
 *   n_out        host: entries written;
 *   bin_offsets  host, n_bins + 1 uint64, or NULL (untouched with
 *                KMC_FLAG_ASCENDING);
 *   stats        host, or NULL.
 * Errors: KMC_ERR_TOO_LARGE, before any device work, when the job's
 * kmc_workspace_size exceeds KMC_STATIC_SCRATCH_BYTES (kmc_last_error states
 * both sizes), and after counting when the table has more than out_cap
 * entries (*n_out then holds the number needed); otherwise as kmc_count_ex.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (each call clears what must start at zero).  Calls that
 * overlapped on one device would race on it: the library serialises the
 * calls of one process on a device with a lock, and each call returns only
 * when its work is done. */
#define KMC_STATIC_SCRATCH_BYTES (256ull << 20)
kmc_status kmc_count_static(kmc_ctx* ctx, const kmc_reads* reads, const kmc_params* params,
                            void* stream, uint64_t* keys_out, uint32_t* counts_out,
                            uint64_t out_cap, uint64_t* n_out, uint64_t* bin_offsets,
                            kmc_stats* stats);

/* ------------------------------------------------------------ database
 * The KMC 2 database (supplement, "Database format" and "API"): the table of
 * a count in the layout of the .kmc_pre / .kmc_suf files, held in device
 * memory, written to and read from those files, and queried in batches on
 * the device.
 *   map       uint32[4^p + 1]: the prefix array of each signature value (the
 *             table's sig_to_bin);
 *   prefixes  n_bins arrays of 4^lut_prefix_length uint64 and a guard:
 *             entry x of array b = index of the first record of bin b whose
 *             k-mer starts with the lut-symbol prefix x; the guard = the
 *             number of records;
 *   records   per table entry (bin by bin, keys ascending inside a bin): the
 *             k - lut_prefix_length symbols after the prefix, four per byte,
 *             leftmost symbol first in the high bits, then the count on
 *             counter_size bytes, least significant byte first (counts above
 *             the field's range are stored as its largest value).
 * .kmc_pre = "KMCP", prefixes, map, header, header size (uint32), "KMCP";
 * .kmc_suf = "KMCS", records, "KMCS"; integers least significant byte first.
 * The header's unused tmp[0] holds `flags` (0 for the paper's canonical,
 * signature-binned database). */
typedef struct kmc_db_info {
  uint32_t kmer_length;
  uint32_t mode;              /* 0: occurrence counters */
  uint32_t counter_size;      /* bytes per counter, 1..4 */
  uint32_t lut_prefix_length; /* symbols cut off as the prefix; 4 | (k - it) */
  uint32_t signature_length;  /* p */
  uint32_t min_count;         /* the count's cutoffs */
  uint32_t max_count;
  uint32_t flags;             /* KMC_FLAG_NON_CANONICAL / KMC_FLAG_PLAIN_MINIMIZERS */
  uint64_t total_kmers;       /* records */
} kmc_db_info;

typedef struct kmc_db kmc_db;

/* Build a database from a bin-major table (host or device; not one counted
 * with KMC_FLAG_ASCENDING) and the parameters it was counted with, on ctx's
 * device.  KMC_ERR_INVALID_ARG if the parameters do not match the table,
 * 4 does not divide k - lut_prefix_len, counter_size is not 1..4, or
 * n_bins * 4^lut_prefix_len exceeds 2^28. */
kmc_status kmc_db_build(kmc_ctx* ctx, const kmc_table* table, const kmc_params* params,
                        uint32_t lut_prefix_len, uint32_t counter_size, kmc_db** out);
/* Header fields of a database. */
kmc_status kmc_db_info_get(const kmc_db* db, kmc_db_info* info);
/* Write <path_prefix>.kmc_pre and <path_prefix>.kmc_suf. */
kmc_status kmc_db_write(const kmc_db* db, const char* path_prefix);
/* Read <path_prefix>.kmc_pre / .kmc_suf into device memory of ctx's device
 * (markers, header position, sizes and prefix arrays checked:
 * KMC_ERR_INVALID_ARG on a malformed file). */
kmc_status kmc_db_open(kmc_ctx* ctx, const char* path_prefix, kmc_db** out);
/* Batched random-access lookup (the API's CheckKmer): kmers = n packed k-mers
 * as read (device memory, key_words per k-mer, hi word first), counts = n
 * uint32 (device memory).  A k-mer is put in canonical form first when the
 * database is canonical; counts[i] = its stored count, or 0 if it is absent
 * or its count lies outside [min_count, max_count] (SetMinCount /
 * SetMaxCount).  On `stream` (NULL = the null stream); returns when done. */
kmc_status kmc_db_query(const kmc_db* db, const uint64_t* kmers, uint64_t n, uint32_t min_count,
                        uint32_t max_count, uint32_t* counts, void* stream);
/* Every record back as (key, count) in database order (the API's listing):
 * keys = total_kmers * key_words uint64, counts = total_kmers uint32, both
 * device memory. */
kmc_status kmc_db_decode(const kmc_db* db, uint64_t* keys, uint32_t* counts, void* stream);
/* Free a database.  NULL is allowed. */
void kmc_db_free(kmc_db* db);

/* -------------------------------------------------------------- parsing
 * FASTQ, FASTA and multi-FASTA text (uncompressed) parsed on the device into
 * CSR reads (the input of the distribution phase, which reads FASTQ / FASTA:
 * Methods, "Sketch of the algorithm"; Additional features).  Lines end with
 * '\n'; a '\r' before it is dropped; the last line may lack the '\n';
 * trailing empty lines are ignored.
 *   FASTQ: records of four lines ('@' header, sequence, '+' line, quality of
 *          the sequence's length); each sequence line is one read.  Wrapped
 *          (multi-line) FASTQ records are not supported.
 *   FASTA: a line starting with '>' opens a record; its read is the
 *          following lines joined without line breaks, up to the next header
 *          (a whole genome record is one long read).
 * Read bytes are copied unchanged (bytes other than A/C/G/T are invalid
 * symbols for the count, as in any read). */
#define KMC_FORMAT_AUTO 0u  /* from the first byte that is not white space */
#define KMC_FORMAT_FASTQ 1u
#define KMC_FORMAT_FASTA 2u
typedef struct kmc_parsed kmc_parsed;
/* Parse n_bytes of text (host memory, or device memory of ctx's device when
 * on_device != 0) on ctx's device.  *reads receives device CSR reads
 * (on_device = 1) owned by *out until kmc_parsed_free.  KMC_ERR_INVALID_ARG
 * for an unknown format, a FASTQ record with a bad '@' or '+' line or a
 * quality line of another length, FASTQ text that ends inside a record, or
 * FASTA sequence before the first header (kmc_last_error names the line). */
kmc_status kmc_parse(kmc_ctx* ctx, const uint8_t* text, uint64_t n_bytes, int32_t on_device,
                     uint32_t format, kmc_reads* reads, kmc_parsed** out);
/* Free parsed reads.  NULL is allowed. */
void kmc_parsed_free(kmc_parsed* parsed);

/* Audit entry (tests): the signature of the window starting at every byte of
 * the input, as the GPU's split kernel computes it, into sig_per_window
 * (host memory, n_bases uint32; 0xFFFFFFFF where no valid k-mer starts), and
 * 1 in superkmer_start (host memory, n_bases bytes; may be NULL) where the
 * kernel opens a new super k-mer.  Signature definition: Methods, "From
 * minimizers to signatures"; super k-mers: Fig. 1.  flags may hold
 * KMC_FLAG_PLAIN_MINIMIZERS. */
kmc_status kmc_debug_signatures(kmc_ctx* ctx, const kmc_reads* reads, uint32_t k, uint32_t p,
                                uint32_t flags, uint32_t* sig_per_window,
                                uint8_t* superkmer_start);

#ifdef __cplusplus
}
#endif

#endif /* KMC_H_ */
