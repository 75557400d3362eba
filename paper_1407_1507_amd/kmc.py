"""Thin ctypes binding of libkmc_hip.so (include/kmc.h).

Argument marshalling only: every step of the counting path runs in the
library's HIP kernels.  Inputs are numpy arrays (host memory) or torch tensors
on a HIP device (device memory); torch is only used for device buffers and
streams.  The library must have been built (``__graft_entry__.build()``); if
it is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmc_hip.so")

KMC_OK = 0
KMC_ERR_INVALID_ARG = 1
KMC_ERR_OUT_OF_MEMORY = 2
KMC_ERR_DEVICE = 3
KMC_ERR_TOO_LARGE = 4
KMC_ERR_BUSY = 5
# device time of each kernel, in the order of kmc_stats.us_kernel
KERNELS = ["sig_hist", "split", "fine_hist", "plan_tiles", "expand_scatter", "tile_sort",
           "big_tiles", "assemble"]
FLAG_DEVICE_TABLE = 0x1
FLAG_PLAIN_MINIMIZERS = 0x2
FLAG_ASCENDING = 0x4
FLAG_NON_CANONICAL = 0x8


def FLAG_KX(x: int) -> int:
    """(k,x)-mers with x = 1..3 (include/kmc.h, KMC_FLAG_KX)."""
    return (x & 3) << 4
FLAG_TEST_NARROW_FINGERPRINT = 0x100  # test only: drives the exact path of 128-bit tiles

EXPORTS = ["kmc_ctx_create", "kmc_ctx_destroy", "kmc_last_error", "kmc_ctx_set_budget", "kmc_count", "kmc_count_ex",
           "kmc_table_free", "kmc_status_str", "kmc_workspace_size", "kmc_count_ws",
           "kmc_batch_count", "kmc_server_start", "kmc_server_submit", "kmc_server_poll",
           "kmc_server_stats_get", "kmc_server_stop", "kmc_debug_signatures",
           "kmc_count_static", "kmc_db_build", "kmc_db_info_get", "kmc_db_write", "kmc_db_open",
           "kmc_db_query", "kmc_db_decode", "kmc_db_free", "kmc_parse", "kmc_parsed_free",
           "kmc_ctx_set_knobs", "kmc_autotune"]
FORMAT_AUTO, FORMAT_FASTQ, FORMAT_FASTA = 0, 1, 2
STATIC_SCRATCH_BYTES = 256 << 20  # KMC_STATIC_SCRATCH_BYTES


class KmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Reads(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n_reads", ctypes.c_uint64), ("n_bases", ctypes.c_uint64),
                ("on_device", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("p", ctypes.c_uint32), ("n_bins", ctypes.c_uint32),
                ("cutoff_min", ctypes.c_uint32), ("cutoff_max", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("counter_max", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "n_reads", "n_bases", "n_kmers", "n_superkmers", "n_distinct", "n_out", "sample_kmers",
        "max_bin_kmers", "n_tiles", "n_big_tiles", "bytes_alg", "split_passes", "n_big_keys",
        "n_big_out", "n_groups", "records_spilled", "n_kx_entries", "n_kx_distinct")] + [
        (n, ctypes.c_double) for n in (
            "us_map", "us_split", "us_expand", "us_sort", "us_assemble", "us_total")] + [
        ("us_kernel", ctypes.c_double * 8), ("us_queue", ctypes.c_double),
        ("us_latency", ctypes.c_double)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "us_kernel"}
        d["us_kernel"] = dict(zip(KERNELS, list(self.us_kernel)))
        return d


class Table(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("key_words", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("keys", ctypes.POINTER(ctypes.c_uint64)),
                ("counts", ctypes.POINTER(ctypes.c_uint32)),
                ("n_bins", ctypes.c_uint32), ("p", ctypes.c_uint32),
                ("bin_offsets", ctypes.POINTER(ctypes.c_uint64)),
                ("sig_to_bin", ctypes.POINTER(ctypes.c_uint32)),
                ("on_device", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("stats", Stats)]


class DbInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "kmer_length", "mode", "counter_size", "lut_prefix_length", "signature_length",
        "min_count", "max_count", "flags")] + [("total_kmers", ctypes.c_uint64)]


class Knobs(ctypes.Structure):
    _fields_ = [("tile_fill", ctypes.c_uint32), ("fine_bits_bias", ctypes.c_int32),
                ("expand_task", ctypes.c_uint32)]


class TuneClass(ctypes.Structure):
    _fields_ = [("key_words", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("sample_bases", ctypes.c_uint64), ("knobs", Knobs), ("pad", ctypes.c_uint32),
                ("us", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_uint32), ("batch_workers", ctypes.c_uint32),
                ("classes", TuneClass * 32)]


# the autotuner's candidate knob sets (tile_fill, fine_bits_bias, expand_task)
KNOB_CANDIDATES = [(3, 0, 0), (2, 0, 0), (3, -1, 0), (3, 1, 0), (3, 0, 512), (3, 0, 1024),
                   (2, 1, 0), (2, 0, 512), (3, 1, 512), (2, -1, 0), (3, -1, 512), (2, 1, 512)]


class Job(ctypes.Structure):
    _fields_ = [("reads", Reads), ("params", Params)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "failed", "admitted_bytes", "peak_admitted_bytes", "budget")] + [
        ("active", ctypes.c_uint32), ("queued", ctypes.c_uint32)]


_lib = None


def _one_hip_runtime():
    """torch ships its own HIP runtime with the same soname as the system's.
    Loading torch first makes the library bind to that already-loaded
    runtime, so one process never holds two HIP runtimes (the second one to
    start would find no GPU)."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _one_hip_runtime()
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.kmc_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        L.kmc_ctx_create.restype = ctypes.c_int
        L.kmc_ctx_destroy.argtypes = [vp]
        L.kmc_ctx_destroy.restype = None
        L.kmc_ctx_set_budget.argtypes = [vp, ctypes.c_uint64]
        L.kmc_ctx_set_budget.restype = ctypes.c_int
        L.kmc_last_error.argtypes = [vp]
        L.kmc_last_error.restype = ctypes.c_char_p
        L.kmc_count.argtypes = [ctypes.POINTER(Reads), ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.POINTER(ctypes.POINTER(Table))]
        L.kmc_count.restype = ctypes.c_int
        L.kmc_count_ex.argtypes = [vp, ctypes.POINTER(Reads), ctypes.POINTER(Params), vp,
                                   ctypes.POINTER(ctypes.POINTER(Table))]
        L.kmc_count_ex.restype = ctypes.c_int
        L.kmc_table_free.argtypes = [ctypes.POINTER(Table)]
        L.kmc_table_free.restype = None
        L.kmc_status_str.argtypes = [ctypes.c_int]
        L.kmc_status_str.restype = ctypes.c_char_p
        L.kmc_debug_signatures.argtypes = [vp, ctypes.POINTER(Reads), ctypes.c_uint32,
                                           ctypes.c_uint32, ctypes.c_uint32, vp, vp]
        L.kmc_debug_signatures.restype = ctypes.c_int
        L.kmc_workspace_size.argtypes = [ctypes.POINTER(Reads), ctypes.POINTER(Params),
                                         ctypes.POINTER(ctypes.c_size_t)]
        L.kmc_workspace_size.restype = ctypes.c_int
        L.kmc_count_ws.argtypes = [vp, ctypes.POINTER(Reads), ctypes.POINTER(Params), vp, vp,
                                   ctypes.c_size_t, ctypes.POINTER(ctypes.POINTER(Table))]
        L.kmc_count_ws.restype = ctypes.c_int
        L.kmc_count_static.argtypes = [vp, ctypes.POINTER(Reads), ctypes.POINTER(Params), vp,
                                       vp, vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                       vp, ctypes.POINTER(Stats)]
        L.kmc_count_static.restype = ctypes.c_int
        L.kmc_db_build.argtypes = [vp, ctypes.POINTER(Table), ctypes.POINTER(Params),
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(vp)]
        L.kmc_db_build.restype = ctypes.c_int
        L.kmc_db_info_get.argtypes = [vp, ctypes.POINTER(DbInfo)]
        L.kmc_db_info_get.restype = ctypes.c_int
        L.kmc_db_write.argtypes = [vp, ctypes.c_char_p]
        L.kmc_db_write.restype = ctypes.c_int
        L.kmc_db_open.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
        L.kmc_db_open.restype = ctypes.c_int
        L.kmc_db_query.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                   vp, vp]
        L.kmc_db_query.restype = ctypes.c_int
        L.kmc_db_decode.argtypes = [vp, vp, vp, vp]
        L.kmc_db_decode.restype = ctypes.c_int
        L.kmc_db_free.argtypes = [vp]
        L.kmc_db_free.restype = None
        L.kmc_parse.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32,
                                ctypes.POINTER(Reads), ctypes.POINTER(vp)]
        L.kmc_parse.restype = ctypes.c_int
        L.kmc_parsed_free.argtypes = [vp]
        L.kmc_parsed_free.restype = None
        L.kmc_ctx_set_knobs.argtypes = [vp, ctypes.POINTER(Knobs)]
        L.kmc_ctx_set_knobs.restype = ctypes.c_int
        L.kmc_autotune.argtypes = [vp, ctypes.POINTER(Job), ctypes.c_uint32,
                                   ctypes.POINTER(TuneReport)]
        L.kmc_autotune.restype = ctypes.c_int
        L.kmc_batch_count.argtypes = [vp, ctypes.POINTER(Job), ctypes.c_uint32,
                                      ctypes.POINTER(ctypes.POINTER(Table))]
        L.kmc_batch_count.restype = ctypes.c_int
        L.kmc_server_start.argtypes = [vp, ctypes.POINTER(ServerCfg), ctypes.POINTER(vp)]
        L.kmc_server_start.restype = ctypes.c_int
        L.kmc_server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]
        L.kmc_server_submit.restype = ctypes.c_int
        L.kmc_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.POINTER(Table))]
        L.kmc_server_poll.restype = ctypes.c_int
        L.kmc_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.kmc_server_stats_get.restype = ctypes.c_int
        L.kmc_server_stop.argtypes = [vp]
        L.kmc_server_stop.restype = None
        _lib = L
    return _lib


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def make_reads(seq, offsets):
    """Reads struct (plus the objects that must stay alive while it is used)."""
    if isinstance(seq, Parsed):
        return seq.reads, (seq,)
    if _is_torch(seq):
        if not (seq.is_cuda and offsets.is_cuda):
            raise ValueError("torch inputs must both live on the GPU")
        if not (seq.is_contiguous() and offsets.is_contiguous()):
            raise ValueError("torch inputs must be contiguous")
        n_reads = offsets.numel() - 1
        r = Reads(seq.data_ptr(), offsets.data_ptr(), n_reads, seq.numel(), 1, 0)
        return r, (seq, offsets)
    seq = np.ascontiguousarray(np.asarray(seq, dtype=np.uint8))
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    if offsets.ndim != 1 or offsets.size < 1:
        raise ValueError("offsets must have n_reads + 1 entries")
    r = Reads(seq.ctypes.data if seq.size else None, offsets.ctypes.data, offsets.size - 1,
              seq.size, 0, 0)
    return r, (seq, offsets)


class Result:
    """A counted table.  Host tables are copied into numpy arrays; device
    tables keep the library's buffers until free() (or garbage collection)."""

    def __init__(self, ptr, keep: bool = False):
        t = ptr.contents
        self.k = t.k
        self.key_words = t.key_words
        self.n = t.n
        self.p = t.p
        self.n_bins = t.n_bins
        self.on_device = bool(t.on_device)
        self.stats = t.stats.as_dict()
        # None in ascending order (entries not grouped by bin)
        self.bin_offsets = (np.ctypeslib.as_array(t.bin_offsets, shape=(t.n_bins + 1,)).copy()
                            if t.bin_offsets else None)
        self.sig_to_bin = np.ctypeslib.as_array(t.sig_to_bin, shape=((1 << (2 * t.p)) + 1,)).copy()
        self._ptr = ptr
        if self.on_device:
            self.keys_ptr = ctypes.cast(t.keys, ctypes.c_void_p).value
            self.counts_ptr = ctypes.cast(t.counts, ctypes.c_void_p).value
            self.keys = self.counts = None
        else:
            n, kw = t.n, t.key_words
            if n:
                keys = np.ctypeslib.as_array(t.keys, shape=(n * kw,)).copy()
                self.counts = np.ctypeslib.as_array(t.counts, shape=(n,)).copy()
            else:
                keys = np.zeros(0, dtype=np.uint64)
                self.counts = np.zeros(0, dtype=np.uint32)
            self.keys = keys.reshape(n, 2) if kw == 2 else keys
            if not keep:  # keep: the library's table stays until free() (kmc_db_build reads it)
                self.free()

    def free(self):
        if self._ptr is not None:
            lib().kmc_table_free(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        st = lib().kmc_ctx_create(device, ctypes.byref(self._h))
        if st != KMC_OK:
            raise KmcError(st, f"kmc_ctx_create: {lib().kmc_status_str(st).decode()}")

    def set_budget(self, device_bytes: int):
        """kmc_ctx_set_budget: device bytes a job's buffers may take (0 = no bound)."""
        st = lib().kmc_ctx_set_budget(self._h, device_bytes)
        if st != KMC_OK:
            raise KmcError(st, "kmc_ctx_set_budget")

    def set_knobs(self, knobs=None):
        """kmc_ctx_set_knobs: (tile_fill, fine_bits_bias, expand_task), or None."""
        k = Knobs(*knobs) if knobs is not None else None
        st = lib().kmc_ctx_set_knobs(self._h, ctypes.byref(k) if k is not None else None)
        if st != KMC_OK:
            raise KmcError(st, "kmc_ctx_set_knobs")

    def autotune(self, jobs) -> dict:
        """kmc_autotune over jobs = [(seq, offsets, params dict), ...]."""
        n = len(jobs)
        arr = (Job * max(n, 1))()
        keep = []
        for i, (seq, off, prm) in enumerate(jobs):
            r, kp = make_reads(seq, off)
            keep.append(kp)
            arr[i].reads = r
            arr[i].params = make_params(**prm)
        rep = TuneReport()
        st = lib().kmc_autotune(self._h, arr, n, ctypes.byref(rep))
        del keep
        if st != KMC_OK:
            self._raise(st, "kmc_autotune")
        return {"batch_workers": rep.batch_workers,
                "classes": [{"key_words": c.key_words, "sample_bases": c.sample_bases,
                             "knobs": (c.knobs.tile_fill, c.knobs.fine_bits_bias,
                                       c.knobs.expand_task), "us": c.us}
                            for c in rep.classes[:rep.n_classes]]}

    def close(self):
        if self._h:
            lib().kmc_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st, what):
        msg = lib().kmc_last_error(self._h).decode()
        raise KmcError(st, f"{what}: {lib().kmc_status_str(st).decode()} {msg}".strip())

    def count(self, seq, offsets, k: int, p: int, n_bins: int, cutoff_min: int = 2,
              cutoff_max: int = 10**9, flags: int = 0, stream=None,
              counter_max: int = 0, keep_table: bool = False) -> Result:
        reads, keep = make_reads(seq, offsets)
        params = make_params(k, p, n_bins, cutoff_min, cutoff_max, flags, counter_max)
        out = ctypes.POINTER(Table)()
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        st = lib().kmc_count_ex(self._h, ctypes.byref(reads), ctypes.byref(params), sp,
                                ctypes.byref(out))
        del keep
        if st != KMC_OK:
            self._raise(st, "kmc_count_ex")
        res = Result(out, keep=keep_table)
        res.params = params
        return res

    def workspace_size(self, seq, offsets, k: int, p: int, n_bins: int, cutoff_min: int = 2,
                       cutoff_max: int = 10**9, flags: int = 0) -> int:
        reads, keep = make_reads(seq, offsets)
        params = make_params(k, p, n_bins, cutoff_min, cutoff_max, flags)
        out = ctypes.c_size_t(0)
        st = lib().kmc_workspace_size(ctypes.byref(reads), ctypes.byref(params), ctypes.byref(out))
        del keep
        if st != KMC_OK:
            raise KmcError(st, f"kmc_workspace_size: {lib().kmc_status_str(st).decode()}")
        return out.value

    def count_ws(self, seq, offsets, k: int, p: int, n_bins: int, cutoff_min: int, cutoff_max: int,
                 workspace, flags: int = 0, stream=None) -> Result:
        """kmc_count_ws: every device buffer of the job is carved from
        `workspace` (a contiguous torch uint8 tensor on the context's device)."""
        reads, keep = make_reads(seq, offsets)
        params = make_params(k, p, n_bins, cutoff_min, cutoff_max, flags)
        out = ctypes.POINTER(Table)()
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        st = lib().kmc_count_ws(self._h, ctypes.byref(reads), ctypes.byref(params), sp,
                                workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                ctypes.byref(out))
        del keep
        if st != KMC_OK:
            self._raise(st, "kmc_count_ws")
        return Result(out)

    def count_static(self, seq, offsets, k: int, p: int, n_bins: int, cutoff_min: int,
                     cutoff_max: int, keys_out, counts_out, flags: int = 0, stream=None):
        """kmc_count_static: the allocation-free count into the caller's device
        buffers keys_out (uint64, n * key_words) and counts_out (int32/uint32,
        n).  Returns (n_out, bin_offsets or None, stats dict)."""
        reads, keep = make_reads(seq, offsets)
        params = make_params(k, p, n_bins, cutoff_min, cutoff_max, flags)
        kw = 1 if k <= 32 else 2
        cap = min(keys_out.numel() // kw, counts_out.numel())
        n_out = ctypes.c_uint64(0)
        bo = np.zeros(n_bins + 1, dtype=np.uint64)
        stats = Stats()
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        st = lib().kmc_count_static(self._h, ctypes.byref(reads), ctypes.byref(params), sp,
                                    keys_out.data_ptr(), counts_out.data_ptr(), cap,
                                    ctypes.byref(n_out), bo.ctypes.data, ctypes.byref(stats))
        del keep
        if st != KMC_OK:
            err = KmcError(st, "kmc_count_static: " + lib().kmc_status_str(st).decode() + " " +
                           lib().kmc_last_error(self._h).decode())
            err.n_out = n_out.value
            raise err
        return n_out.value, (None if flags & FLAG_ASCENDING else bo), stats.as_dict()

    def batch_count(self, jobs) -> list:
        """kmc_batch_count over jobs = [(seq, offsets, params dict), ...];
        params keys: k, p, n_bins, cutoff_min, cutoff_max[, flags]."""
        n = len(jobs)
        arr = (Job * max(n, 1))()
        keep = []
        for i, (seq, off, prm) in enumerate(jobs):
            r, kp = make_reads(seq, off)
            keep.append(kp)
            arr[i].reads = r
            arr[i].params = make_params(**prm)
        outs = (ctypes.POINTER(Table) * max(n, 1))()
        st = lib().kmc_batch_count(self._h, arr, n, outs)
        del keep
        if st != KMC_OK:
            self._raise(st, "kmc_batch_count")
        return [Result(outs[i]) for i in range(n)]

    def debug_signatures(self, seq, offsets, k: int, p: int, flags: int = 0):
        reads, keep = make_reads(seq, offsets)
        nb = int(reads.n_bases)
        sig = np.zeros(max(nb, 1), dtype=np.uint32)
        start = np.zeros(max(nb, 1), dtype=np.uint8)
        st = lib().kmc_debug_signatures(self._h, ctypes.byref(reads), k, p, flags,
                                        sig.ctypes.data, start.ctypes.data)
        del keep
        if st != KMC_OK:
            self._raise(st, "kmc_debug_signatures")
        return sig[:nb], start[:nb]


class Parsed:
    """Reads parsed on the device from FASTQ / FASTA text (kmc_parse); pass it
    as `seq` (offsets None) to Context.count."""

    def __init__(self, ctx: "Context", text, fmt: int = FORMAT_AUTO):
        self._h = ctypes.c_void_p()
        self.reads = Reads()
        if _is_torch(text):
            ptr, n, on_dev = text.data_ptr(), text.numel(), 1
            keep = text
        else:
            keep = np.frombuffer(bytes(text), dtype=np.uint8) if not isinstance(
                text, np.ndarray) else np.ascontiguousarray(text, dtype=np.uint8)
            ptr, n, on_dev = (keep.ctypes.data if keep.size else None), keep.size, 0
        st = lib().kmc_parse(ctx._h, ptr, n, on_dev, fmt, ctypes.byref(self.reads),
                             ctypes.byref(self._h))
        del keep
        if st != KMC_OK:
            ctx._raise(st, "kmc_parse")
        self.n_reads = self.reads.n_reads
        self.n_bases = self.reads.n_bases

    def to_host(self):
        """(seq, offsets) copied to numpy arrays."""
        hip = ctypes.CDLL("libamdhip64.so")
        seq = np.zeros(self.n_bases, dtype=np.uint8)
        off = np.zeros(self.n_reads + 1, dtype=np.uint64)
        if self.n_bases:
            assert hip.hipMemcpy(ctypes.c_void_p(seq.ctypes.data), ctypes.c_void_p(self.reads.seq),
                                 ctypes.c_size_t(seq.nbytes), 2) == 0
        assert hip.hipMemcpy(ctypes.c_void_p(off.ctypes.data), ctypes.c_void_p(self.reads.offsets),
                             ctypes.c_size_t(off.nbytes), 2) == 0
        return seq, off

    def free(self):
        if self._h:
            lib().kmc_parsed_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Db:
    """A KMC 2 database in device memory (kmc_db_*): built from a counted
    table (Result of Context.count with keep_table=True or a device table),
    or opened from .kmc_pre / .kmc_suf files."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        info = DbInfo()
        st = lib().kmc_db_info_get(self._h, ctypes.byref(info))
        if st != KMC_OK:
            raise KmcError(st, "kmc_db_info_get")
        self.info = {n: getattr(info, n) for n, _ in info._fields_}
        self.key_words = 1 if info.kmer_length <= 32 else 2

    @classmethod
    def build(cls, ctx: "Context", table: "Result", lut_prefix_len: int, counter_size: int = 4):
        if table._ptr is None:
            raise ValueError("the table was freed; count with keep_table=True")
        h = ctypes.c_void_p()
        st = lib().kmc_db_build(ctx._h, table._ptr, ctypes.byref(table.params), lut_prefix_len,
                                counter_size, ctypes.byref(h))
        if st != KMC_OK:
            ctx._raise(st, "kmc_db_build")
        return cls(h)

    @classmethod
    def open(cls, ctx: "Context", path_prefix: str):
        h = ctypes.c_void_p()
        st = lib().kmc_db_open(ctx._h, path_prefix.encode(), ctypes.byref(h))
        if st != KMC_OK:
            ctx._raise(st, "kmc_db_open")
        return cls(h)

    def write(self, path_prefix: str):
        st = lib().kmc_db_write(self._h, path_prefix.encode())
        if st != KMC_OK:
            raise KmcError(st, f"kmc_db_write: {lib().kmc_status_str(st).decode()}")

    def query(self, kmers, counts_out, min_count: int = 0, max_count: int = 2**32 - 1,
              stream=None):
        """kmers: torch uint64/int64 tensor on the device (n * key_words);
        counts_out: torch int32 tensor of n entries on the device."""
        n = kmers.numel() // self.key_words
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        st = lib().kmc_db_query(self._h, kmers.data_ptr(), n, min_count, max_count,
                                counts_out.data_ptr(), sp)
        if st != KMC_OK:
            raise KmcError(st, f"kmc_db_query: {lib().kmc_status_str(st).decode()}")

    def decode(self, keys_out, counts_out, stream=None):
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        st = lib().kmc_db_decode(self._h, keys_out.data_ptr(), counts_out.data_ptr(), sp)
        if st != KMC_OK:
            raise KmcError(st, f"kmc_db_decode: {lib().kmc_status_str(st).decode()}")

    def free(self):
        if self._h:
            lib().kmc_db_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def make_params(k: int, p: int, n_bins: int, cutoff_min: int = 2, cutoff_max: int = 10**9,
                flags: int = 0, counter_max: int = 0) -> Params:
    return Params(k, p, n_bins, cutoff_min, min(cutoff_max, 2**32 - 1), flags, counter_max)


class Server:
    """kmc_server_*: jobs submitted while others run, admitted by their HBM
    footprint against `hbm_budget` bytes (0 = 90% of free device memory), at
    most `max_active` at once (0 = 4)."""

    def __init__(self, ctx: Context, hbm_budget: int = 0, max_active: int = 0):
        self._h = ctypes.c_void_p()
        self._keep = {}
        cfg = ServerCfg(hbm_budget, max_active, 0)
        st = lib().kmc_server_start(ctx._h, ctypes.byref(cfg), ctypes.byref(self._h))
        if st != KMC_OK:
            raise KmcError(st, f"kmc_server_start: {lib().kmc_status_str(st).decode()}")

    def submit(self, seq, offsets, k: int, p: int, n_bins: int, cutoff_min: int = 2,
               cutoff_max: int = 10**9, flags: int = 0) -> int:
        reads, keep = make_reads(seq, offsets)
        job = Job(reads, make_params(k, p, n_bins, cutoff_min, cutoff_max, flags))
        t = ctypes.c_uint64(0)
        st = lib().kmc_server_submit(self._h, ctypes.byref(job), ctypes.byref(t))
        if st != KMC_OK:
            raise KmcError(st, f"kmc_server_submit: {lib().kmc_status_str(st).decode()}")
        self._keep[t.value] = keep  # the reads stay borrowed until polled
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """The job's Result, or None if it is not done and wait is False."""
        out = ctypes.POINTER(Table)()
        st = lib().kmc_server_poll(self._h, ticket, 1 if wait else 0, ctypes.byref(out))
        if st == KMC_ERR_BUSY and not wait:
            return None
        self._keep.pop(ticket, None)
        if st != KMC_OK:
            raise KmcError(st, f"kmc_server_poll: {lib().kmc_status_str(st).decode()}")
        return Result(out)

    def stats(self) -> dict:
        s = ServerStats()
        st = lib().kmc_server_stats_get(self._h, ctypes.byref(s))
        if st != KMC_OK:
            raise KmcError(st, "kmc_server_stats_get")
        return {n: getattr(s, n) for n, _ in s._fields_}

    def stop(self):
        if self._h:
            lib().kmc_server_stop(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def count(seq, offsets, k: int, p: int, n_bins: int, cutoff_min: int = 2,
          cutoff_max: int = 10**9) -> Result:
    """kmc_count on the calling thread's default context (device 0)."""
    reads, keep = make_reads(seq, offsets)
    out = ctypes.POINTER(Table)()
    st = lib().kmc_count(ctypes.byref(reads), k, p, n_bins, cutoff_min,
                         min(cutoff_max, 2**32 - 1), ctypes.byref(out))
    del keep
    if st != KMC_OK:
        raise KmcError(st, f"kmc_count: {lib().kmc_status_str(st).decode()}")
    return Result(out)
