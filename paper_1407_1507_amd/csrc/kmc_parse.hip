// Input records on the device: FASTQ, FASTA and multi-FASTA text parsed into
// the library's CSR reads (the step before the distribution phase, which in
// the paper reads FASTQ / FASTA files: Methods, "Sketch of the algorithm";
// Additional features).  Compressed input is decompressed on the host.
//
// Lines end with '\n' (a '\r' before it is dropped; the last line may lack
// the '\n').  FASTQ: records of four lines, '@' header, sequence, '+' line,
// quality of the sequence's length; the sequence line is the read.  FASTA:
// a line starting with '>' opens a record; the record's read is its
// following lines joined without line breaks, up to the next header.  The
// read bytes are copied as they are (bytes other than A/C/G/T are invalid
// symbols for the count, as in any read).
//
// Passes: newlines counted per chunk, a scan, newline positions written in
// order; one thread per line classifies it and takes its sequence length; a
// scan of the lengths gives each sequence line's place in the output and each
// read's offset; one wavefront per line copies its bytes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/kmc.h"
#include "kmc_device.h"
#include "kmc_internal.h"

using namespace kmc;

struct kmc_parsed {
  int device = 0;
  uint8_t* seq = nullptr;      // device, n_bases (+ 16 bytes of slack)
  uint64_t* offsets = nullptr; // device, n_reads + 1
  uint64_t n_reads = 0, n_bases = 0;
};

namespace {

constexpr uint32_t kChunk = 16384;       // bytes per newline-counting workgroup
constexpr uint32_t kPerThread = kChunk / 256;

// Bytes equal to '\n' in a 32-bit word: a zero-byte test on w ^ 0x0A0A0A0A
// (each 0x80 bit marks a zero byte; the carry-free form, exact for every
// byte).
__device__ __forceinline__ uint32_t nl_mask(uint32_t w) {
  const uint32_t x = w ^ 0x0A0A0A0Au;
  return ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
}

// The 16 bytes at chunk offset q (q % 16 == 0) of the text, as four words;
// bytes at or past n read as 0.
__device__ __forceinline__ uint4 load16(const uint8_t* __restrict__ t, uint64_t n, bool a16,
                                        uint64_t x) {
  if (a16 && x + 16 <= n) return *reinterpret_cast<const uint4*>(t + x);
  uint32_t w[4] = {0, 0, 0, 0};
  for (int i = 0; i < 16; ++i)
    if (x + i < n) w[i >> 2] |= (uint32_t)t[x + i] << (8 * (i & 3));
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Newlines of chunk c (kChunk bytes) into cnt[c]: each thread counts its
// kPerThread consecutive bytes, 16 at a time.
__global__ void __launch_bounds__(256)
k_nl_count(const uint8_t* __restrict__ t, uint64_t n, bool a16, uint32_t* cnt) {
  const uint64_t x0 = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kPerThread;
  uint32_t m = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPerThread; q += 16) {
    const uint4 v = load16(t, n, a16, x0 + q);
    m += __popc(nl_mask(v.x)) + __popc(nl_mask(v.y)) + __popc(nl_mask(v.z)) +
         __popc(nl_mask(v.w));
  }
  for (int d = 32; d >= 1; d >>= 1) m += __shfl_xor(m, d, 64);
  __shared__ uint32_t w[4];
  if ((threadIdx.x & 63u) == 0) w[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = w[0] + w[1] + w[2] + w[3];
}

// Positions of the newlines of chunk c in order, from nl_base[c]: each thread
// takes kPerThread consecutive bytes; a block scan orders the threads.
__global__ void __launch_bounds__(256)
k_nl_emit(const uint8_t* __restrict__ t, uint64_t n, bool a16,
          const uint64_t* __restrict__ nl_base, uint64_t* pos) {
  __shared__ uint32_t tmp[4];
  const uint64_t x0 = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kPerThread;
  uint4 v[kPerThread / 16];
  uint32_t m = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPerThread / 16; ++q) {
    v[q] = load16(t, n, a16, x0 + 16 * q);
    m += __popc(nl_mask(v[q].x)) + __popc(nl_mask(v[q].y)) + __popc(nl_mask(v[q].z)) +
         __popc(nl_mask(v[q].w));
  }
  uint32_t total;
  const uint32_t before = block_scan_one(m, tmp, total);
  uint64_t o = nl_base[blockIdx.x] + before;
#pragma unroll
  for (uint32_t q = 0; q < kPerThread / 16; ++q) {
    const uint32_t words[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
    for (int wi = 0; wi < 4; ++wi) {
      uint32_t mk = nl_mask(words[wi]);
      while (mk) {
        const uint32_t bit = __ffs(mk) - 1;  // 8 * byte + 7
        pos[o++] = x0 + 16 * q + 4 * wi + (bit >> 3);
        mk &= mk - 1;
      }
    }
  }
}

struct Lines {
  const uint8_t* t;
  const uint64_t* nl;  // newline positions
  uint64_t n_nl, n_bytes, n_lines;
  __device__ void span(uint64_t i, uint64_t& b, uint64_t& e) const {
    b = i == 0 ? 0 : nl[i - 1] + 1;
    e = i < n_nl ? nl[i] : n_bytes;
    if (e > b && t[e - 1] == '\r') --e;
  }
};

// *last = 1 + index of the last line that holds anything (trailing empty
// lines carry nothing and are dropped).  One wavefront walks back from the
// end, 64 lines a step, for at most kLastSteps steps (trailing empty lines
// are few); if all of those are empty it leaves ~0 and the host runs
// k_last_line_all.
constexpr uint32_t kLastSteps = 64;
__global__ void __launch_bounds__(64)
k_last_line(Lines L, unsigned long long* last) {
  const uint32_t lane = threadIdx.x;
  uint64_t top = L.n_lines;
  for (uint32_t step = 0; step < kLastSteps && top > 0; ++step) {
    bool ne = false;
    if (lane < top) {  // lane l tests line top - 1 - l
      uint64_t b, e;
      L.span(top - 1 - lane, b, e);
      ne = e > b;
    }
    const uint64_t m = __ballot(ne);
    if (m) {  // the lowest such lane holds the highest non-empty line
      if (lane == 0) *last = top - (uint64_t)(__ffsll((unsigned long long)m) - 1);
      return;
    }
    top = top > 64 ? top - 64 : 0;
  }
  if (lane == 0) *last = top == 0 ? 0ull : ~0ull;
}
// The same over every line (one atomic per wavefront).
__global__ void __launch_bounds__(256)
k_last_line_all(Lines L, unsigned long long* last) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ne = false;
  if (i < L.n_lines) {
    uint64_t b, e;
    L.span(i, b, e);
    ne = e > b;
  }
  const uint64_t m = __ballot(ne);
  if (m && (threadIdx.x & 63u) == 0) {
    const uint64_t w0 = i;  // line of lane 0
    atomicMax(last, (unsigned long long)(w0 + 64 - __clzll((long long)m)));
  }
}

// Per line: its sequence length (0 for header, '+' and quality lines) and,
// in hdr, 1 where a read starts.  FASTQ checks go to err (smallest bad line).
__global__ void __launch_bounds__(256)
k_lines(Lines L, uint32_t fastq, uint32_t* len, uint32_t* starts,
        unsigned long long* err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n_lines) return;
  uint64_t b, e;
  L.span(i, b, e);
  const uint64_t n = e - b;
  const uint8_t first = n ? L.t[b] : 0;
  uint32_t l = 0, st = 0;
  bool bad = n >= (1ull << 32);
  if (fastq) {
    switch (i & 3) {
      case 0: bad = bad || first != '@'; break;
      case 1: l = (uint32_t)n; st = 1; break;
      case 2: bad = bad || first != '+'; break;
      default: {
        uint64_t sb, se;
        L.span(i - 2, sb, se);
        bad = bad || (se - sb) != n;
      }
    }
  } else if (first == '>') {
    st = 1;
  } else {
    l = (uint32_t)n;
    // sequence text before the first header
    bad = bad || (n && i == 0);
  }
  len[i] = l;
  starts[i] = st;
  if (bad) atomicMin(err, (unsigned long long)i);
}

// Read offsets: FASTQ read r is line 4r + 1; a FASTA read starts at its
// header line (its rank among headers from the scan of starts).
__global__ void __launch_bounds__(256)
k_offsets(uint64_t n_lines, const uint32_t* __restrict__ starts,
          const uint64_t* __restrict__ start_rank, const uint64_t* __restrict__ out_pos,
          uint64_t* offsets) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_lines) return;
  if (i == n_lines) {
    offsets[start_rank[n_lines]] = out_pos[n_lines];
    return;
  }
  if (starts[i]) offsets[start_rank[i]] = out_pos[i];
}

// One wavefront per line: copy its sequence bytes to their place.
__global__ void __launch_bounds__(256)
k_copy(Lines L, const uint32_t* __restrict__ len, const uint64_t* __restrict__ out_pos,
       uint8_t* seq) {
  // one wavefront per 64 consecutive lines: the lines that hold sequence
  // are copied one after another, 64 bytes at a time
  const uint64_t i0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64;
  const uint32_t lane = threadIdx.x & 63u;
  if (i0 >= L.n_lines) return;
  // each lane loads its own line's length, start and output position, so
  // the copies below wait on no per-line load
  const uint32_t my_len = i0 + lane < L.n_lines ? len[i0 + lane] : 0u;
  unsigned long long my_b = 0, my_o = 0;
  if (my_len) {
    uint64_t b, e;
    L.span(i0 + lane, b, e);
    my_b = b;
    my_o = out_pos[i0 + lane];
  }
  uint64_t m = __ballot(my_len != 0);
  while (m) {
    const int l = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const uint32_t n = (uint32_t)__shfl((int)my_len, l);
    const uint64_t b = __shfl(my_b, l), o = __shfl(my_o, l);
    for (uint32_t j = lane; j < n; j += 64) seq[o + j] = L.t[b + j];
  }
}

uint32_t grid(uint64_t n) { return (uint32_t)((n + 255) / 256); }

// Scratch of a parse: the context's cached buffers (slot per array), so that
// repeated parses allocate nothing.
struct Scratch {
  kmc_ctx* c;
  int next = 0;
  template <class T>
  T* get(size_t n) {
    return static_cast<T*>(ctx_aux_buffer(c, next++, std::max<size_t>(n, 1) * sizeof(T)));
  }
};

}  // namespace

extern "C" {

kmc_status kmc_parse(kmc_ctx* ctx, const uint8_t* text, uint64_t n_bytes, int32_t on_device,
                     uint32_t format, kmc_reads* reads, kmc_parsed** out) {
  if (!out || !reads) return KMC_ERR_INVALID_ARG;
  *out = nullptr;
  std::memset(reads, 0, sizeof(*reads));
  if (!ctx || (n_bytes && !text) || format > KMC_FORMAT_FASTA) return KMC_ERR_INVALID_ARG;
  const int dev = ctx_device(ctx);
  if (hipSetDevice(dev) != hipSuccess) {
    (void)hipGetLastError();
    return KMC_ERR_DEVICE;
  }
  hipStream_t s = ctx_stream(ctx);
  Scratch S{ctx};
  auto dev_err = [&](const char* what) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    ctx_set_error(ctx, what);
    return KMC_ERR_DEVICE;
  };
  const uint8_t* t = text;
  if (!on_device && n_bytes) {
    uint8_t* d = S.get<uint8_t>(n_bytes);
    if (!d) return KMC_ERR_OUT_OF_MEMORY;
    if (hipMemcpyAsync(d, text, n_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
      return dev_err("H2D of the text failed");
    t = d;
  }
  // the format from the first byte that is not white space
  uint32_t fmt = format;
  if (fmt == KMC_FORMAT_AUTO) {
    uint8_t head[256];
    const uint64_t nh = n_bytes < sizeof(head) ? n_bytes : sizeof(head);
    if (nh && hipMemcpyAsync(head, t, nh, hipMemcpyDeviceToHost, s) != hipSuccess)
      return dev_err("D2H failed");
    if (hipStreamSynchronize(s) != hipSuccess) return dev_err("sync failed");
    for (uint64_t i = 0; i < nh && fmt == KMC_FORMAT_AUTO; ++i) {
      if (head[i] == '@') fmt = KMC_FORMAT_FASTQ;
      else if (head[i] == '>') fmt = KMC_FORMAT_FASTA;
      else if (head[i] != '\n' && head[i] != '\r' && head[i] != ' ' && head[i] != '\t') break;
    }
    if (fmt == KMC_FORMAT_AUTO && nh) {
      ctx_set_error(ctx, "input is neither FASTQ ('@') nor FASTA ('>')");
      return KMC_ERR_INVALID_ARG;
    }
    if (fmt == KMC_FORMAT_AUTO) fmt = KMC_FORMAT_FASTA;  // empty input: no reads
  }
  // newline positions
  const bool a16 = ((uintptr_t)t & 15u) == 0;
  const uint64_t n_chunks = (n_bytes + kChunk - 1) / kChunk;
  uint32_t* cnt = S.get<uint32_t>(n_chunks);
  uint64_t* nl_base = S.get<uint64_t>(n_chunks + 1);
  uint64_t* scan_tmp = S.get<uint64_t>(scan_tmp_words(n_chunks));
  if (!cnt || !nl_base || !scan_tmp) return KMC_ERR_OUT_OF_MEMORY;
  if (n_chunks)
    hipLaunchKernelGGL(k_nl_count, dim3((uint32_t)n_chunks), dim3(256), 0, s, t, n_bytes, a16,
                       cnt);
  if (launch_scan_u32(s, cnt, n_chunks, nl_base, scan_tmp) != hipSuccess)
    return dev_err("newline scan failed");
  uint64_t n_nl = 0;
  uint8_t last = '\n';
  if (hipMemcpyAsync(&n_nl, nl_base + n_chunks, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      (n_bytes && hipMemcpyAsync(&last, t + n_bytes - 1, 1, hipMemcpyDeviceToHost, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return dev_err("newline count failed");
  uint64_t* nl = S.get<uint64_t>(n_nl);
  if (!nl) return KMC_ERR_OUT_OF_MEMORY;
  if (n_chunks)
    hipLaunchKernelGGL(k_nl_emit, dim3((uint32_t)n_chunks), dim3(256), 0, s, t, n_bytes, a16,
                       nl_base, nl);
  // lines: one per newline, plus an unterminated last line; trailing empty
  // lines are dropped
  uint64_t n_lines = n_nl + ((n_bytes && last != '\n') ? 1 : 0);
  unsigned long long* err = S.get<unsigned long long>(2);
  if (!err) return KMC_ERR_OUT_OF_MEMORY;
  const unsigned long long init[2] = {~0ull, 0ull};  // smallest bad line, last line
  if (hipMemcpyAsync(err, init, 16, hipMemcpyHostToDevice, s) != hipSuccess)
    return dev_err("H2D failed");
  if (n_lines) {
    const Lines L0{t, nl, n_nl, n_bytes, n_lines};
    hipLaunchKernelGGL(k_last_line, dim3(1), dim3(64), 0, s, L0, err + 1);
    unsigned long long lastne = 0;
    if (hipMemcpyAsync(&lastne, err + 1, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return dev_err("line scan failed");
    if (lastne == ~0ull) {  // more than kLastSteps * 64 empty lines at the end
      const unsigned long long zero = 0;
      if (hipMemcpyAsync(err + 1, &zero, 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return dev_err("H2D failed");
      hipLaunchKernelGGL(k_last_line_all, dim3(grid(n_lines)), dim3(256), 0, s, L0, err + 1);
      if (hipMemcpyAsync(&lastne, err + 1, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return dev_err("line scan failed");
    }
    n_lines = lastne;
  }
  if (fmt == KMC_FORMAT_FASTQ && n_lines % 4 != 0) {
    ctx_set_error(ctx, ("FASTQ input ends inside a record (" + std::to_string(n_lines) +
                        " lines)").c_str());
    return KMC_ERR_INVALID_ARG;
  }
  uint32_t* len = S.get<uint32_t>(n_lines);
  uint32_t* starts = S.get<uint32_t>(n_lines);
  uint64_t* out_pos = S.get<uint64_t>(n_lines + 1);
  uint64_t* rank = S.get<uint64_t>(n_lines + 1);
  uint64_t* scan2 = S.get<uint64_t>(scan_tmp_words(n_lines));
  if (!len || !starts || !out_pos || !rank || !scan2) return KMC_ERR_OUT_OF_MEMORY;
  const unsigned long long none = ~0ull;
  const Lines L{t, nl, n_nl, n_bytes, n_lines};
  if (n_lines)
    hipLaunchKernelGGL(k_lines, dim3(grid(n_lines)), dim3(256), 0, s, L,
                       fmt == KMC_FORMAT_FASTQ ? 1u : 0u, len, starts, err);
  if (launch_scan_u32(s, len, n_lines, out_pos, scan2) != hipSuccess ||
      launch_scan_u32(s, starts, n_lines, rank, scan2) != hipSuccess)
    return dev_err("line scans failed");
  unsigned long long bad = 0;
  uint64_t sums[2] = {0, 0};
  if (hipMemcpyAsync(&bad, err, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&sums[0], out_pos + n_lines, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&sums[1], rank + n_lines, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return dev_err("parse kernels failed");
  if (bad != none) {
    ctx_set_error(ctx, ((fmt == KMC_FORMAT_FASTQ ? "malformed FASTQ record at line "
                                                 : "FASTA sequence before a header at line ") +
                        std::to_string(bad + 1)).c_str());
    return KMC_ERR_INVALID_ARG;
  }
  kmc_parsed* P = new (std::nothrow) kmc_parsed();
  if (!P) return KMC_ERR_OUT_OF_MEMORY;
  P->device = dev;
  P->n_bases = sums[0];
  P->n_reads = sums[1];
  if (hipMalloc(&P->seq, P->n_bases + 16) != hipSuccess ||
      hipMalloc(&P->offsets, (P->n_reads + 1) * 8) != hipSuccess) {
    (void)hipGetLastError();
    kmc_parsed_free(P);
    return KMC_ERR_OUT_OF_MEMORY;
  }
  if (n_lines) {
    hipLaunchKernelGGL(k_offsets, dim3(grid(n_lines + 1)), dim3(256), 0, s, n_lines, starts, rank,
                       out_pos, P->offsets);
    hipLaunchKernelGGL(k_copy, dim3(grid((n_lines + 63) / 64 * 64)), dim3(256), 0, s, L, len,
                       out_pos, P->seq);
  } else if (hipMemsetAsync(P->offsets, 0, 8, s) != hipSuccess) {
    kmc_parsed_free(P);
    return dev_err("memset failed");
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    kmc_parsed_free(P);
    return dev_err("parse copy failed");
  }
  reads->seq = P->seq;
  reads->offsets = P->offsets;
  reads->n_reads = P->n_reads;
  reads->n_bases = P->n_bases;
  reads->on_device = 1;
  *out = P;
  return KMC_OK;
}

void kmc_parsed_free(kmc_parsed* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->seq) (void)hipFree(p->seq);
  if (p->offsets) (void)hipFree(p->offsets);
  delete p;
}

}  // extern "C"
