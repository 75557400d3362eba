"""The KMC 2 database layout (supplement, "Database format") and its batched
device lookup (supplement, "API": CheckKmer, SetMinCount / SetMaxCount) and
listing (ReadNextKmer).

The .kmc_pre / .kmc_suf files the library writes are parsed here by a plain
reader that follows the supplement's description (markers, header position
8 bytes from the end, header, prefix arrays, map; suffix records of
(k - lut) / 4 bytes plus counter_size bytes), and every record is checked
against the oracle's table; lookups are checked against the oracle's counts.
The supplement's own examples pin the layout: the signature ACGAC = 97 of
ATACGACAAATG picks map entry 97, its prefix ATAC = 49 picks the record range,
and CCACAAAT packs as 0x51 0x03."""
import ctypes
import os
import struct

import numpy as np
import pytest

import oracle
from oracle import strings as S
from paper_1407_1507_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kmc():
    from paper_1407_1507_amd import kmc as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(kmc):
    c = kmc.Context(0)
    yield c
    c.close()


def to_reads(strs):
    seq = np.frombuffer("".join(strs).encode(), dtype=np.uint8).copy()
    off = np.zeros(len(strs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in strs])
    return seq, off


def read_db(prefix):
    """Parse the two files as the supplement describes them."""
    pre = open(prefix + ".kmc_pre", "rb").read()
    suf = open(prefix + ".kmc_suf", "rb").read()
    assert pre[:4] == b"KMCP" and pre[-4:] == b"KMCP"
    assert suf[:4] == b"KMCS" and suf[-4:] == b"KMCS"
    x = struct.unpack_from("<I", pre, len(pre) - 8)[0]
    h0 = len(pre) - (x + 8)
    k, mode, cs, lut, sig_len, cmin, cmax = struct.unpack_from("<7I", pre, h0)
    total = struct.unpack_from("<Q", pre, h0 + 28)[0]
    tmp = struct.unpack_from("<7I", pre, h0 + 36)
    ver = struct.unpack_from("<I", pre, h0 + 64)[0]
    n_sig = 4 ** sig_len + 1
    map_off = h0 - 4 * n_sig
    sig_map = np.frombuffer(pre, dtype="<u4", count=n_sig, offset=map_off)
    n_pre = (map_off - 4) // 8
    prefixes = np.frombuffer(pre, dtype="<u8", count=n_pre, offset=4)
    sb = (k - lut) // 4
    rb = sb + cs
    body = np.frombuffer(suf, dtype=np.uint8, count=len(suf) - 8, offset=4)
    assert body.size == total * rb
    recs = body.reshape(total, rb) if total else body.reshape(0, rb)
    return dict(k=k, mode=mode, cs=cs, lut=lut, sig_len=sig_len, cmin=cmin, cmax=cmax,
                total=total, tmp=tmp, ver=ver, map=sig_map, prefixes=prefixes, recs=recs,
                sb=sb, raw_pre=pre)


def db_entries(d):
    """(key, count) of every record, from its prefix array slot and suffix."""
    k, lut, sb, cs = d["k"], d["lut"], d["sb"], d["cs"]
    L = 4 ** lut
    pre = [int(v) for v in d["prefixes"]]
    out = []
    slot = 0
    for r in range(d["total"]):
        while pre[slot + 1] <= r:
            slot += 1
        x = slot % L
        rec = d["recs"][r]
        suffix = int.from_bytes(bytes(rec[:sb]), "big")
        count = int.from_bytes(bytes(rec[sb:sb + cs]), "little")
        out.append(((x << (2 * (k - lut))) | suffix, count, slot // L))
    return out


def lookup(d, key, p, flt=True):
    """The supplement's lookup: signature -> map -> prefix array, prefix ->
    record range, binary search of the suffix."""
    k, lut, sb, cs = d["k"], d["lut"], d["sb"], d["cs"]
    s = "".join("ACGT"[(key >> (2 * (k - 1 - t))) & 3] for t in range(k))
    sig_s = S.signature(s, p, flt)
    sig = S.encode(sig_s) if sig_s is not None else 4 ** p
    arr = int(d["map"][sig])
    x = key >> (2 * (k - lut)) if lut else 0
    lo = int(d["prefixes"][arr * 4 ** lut + x])
    hi = int(d["prefixes"][arr * 4 ** lut + x + 1])
    want = key & ((1 << (2 * (k - lut))) - 1)
    while lo < hi:
        mid = (lo + hi) // 2
        rec = d["recs"][mid]
        v = int.from_bytes(bytes(rec[:sb]), "big")
        if v == want:
            return int.from_bytes(bytes(rec[sb:sb + cs]), "little")
        if v < want:
            lo = mid + 1
        else:
            hi = mid
    return 0


def as_ints(keys):
    if keys.ndim == 2:
        return [(int(a) << 64) | int(b) for a, b in keys]
    return [int(a) for a in keys]


def revcomp_int(key, k):
    r = 0
    for t in range(k):
        r = r * 4 + (3 - ((key >> (2 * t)) & 3))
    return r


def pack_queries(ints, k):
    import torch
    if k <= 32:
        a = np.array(ints, dtype=np.uint64)
    else:
        a = np.array([[v >> 64, v & (2**64 - 1)] for v in ints], dtype=np.uint64).reshape(-1)
    return torch.from_numpy(a.view(np.int64)).to("cuda:0")


@pytest.mark.parametrize("name,scale,lut,cs", [
    ("genome-5M-2Mx100", 0.01, 4, 4), ("genome-5M-2Mx100", 0.01, 0, 1),
    ("genome-5M-2Mx100", 0.01, 8, 2), ("repeats-50M-30x150-k55", 0.002, 3, 3),
    ("repeats-50M-30x150-k55", 0.002, 7, 1)])
def test_db_files_match_oracle(ctx, kmc, tmp_path, name, scale, lut, cs):
    seq, off, p = synth.make(name, scale)
    k = p["k"]
    res = ctx.count(seq, off, k, p["p"], p["n_bins"], p["cutoff_min"], p["cutoff_max"],
                    keep_table=True)
    db = kmc.Db.build(ctx, res, lut, cs)
    path = str(tmp_path / "db")
    db.write(path)
    d = read_db(path)
    assert (d["k"], d["mode"], d["cs"], d["lut"], d["sig_len"]) == (k, 0, cs, lut, p["p"])
    assert (d["cmin"], d["cmax"], d["total"], d["ver"]) == (p["cutoff_min"], p["cutoff_max"],
                                                            res.n, 0x200)
    assert d["tmp"][0] == 0  # canonical, signatures: the paper's own database
    assert np.array_equal(d["map"], res.sig_to_bin)
    assert len(d["prefixes"]) == p["n_bins"] * 4 ** lut + 1
    ent = db_entries(d)
    ok_keys, ok_counts = oracle.count(seq, off, k, p["cutoff_min"], p["cutoff_max"])
    cap = 2 ** (8 * cs) - 1
    want = dict(zip(as_ints(ok_keys), (min(int(c), cap) for c in ok_counts)))
    assert len(ent) == len(want)
    assert {e[0]: e[1] for e in ent} == want
    # records of one prefix array lie in its bin, keys ascending inside it
    sig = oracle.key_signatures(ok_keys, k, p["p"])
    bin_of = dict(zip(as_ints(ok_keys), (int(res.sig_to_bin[s]) for s in sig)))
    assert all(bin_of[key] == b for key, _, b in ent)
    assert all(ent[i][2] < ent[i + 1][2] or ent[i][0] < ent[i + 1][0]
               for i in range(len(ent) - 1))
    # the supplement's lookup on the file finds sampled keys and misses others
    rng = np.random.default_rng(lut)
    for key in rng.choice(list(want), 200, replace=False):
        assert lookup(d, int(key), p["p"]) == want[int(key)]
    res.free()
    db.free()


def test_db_query_matches_oracle(ctx, kmc):
    import torch
    for name, scale in (("genome-5M-2Mx100", 0.02), ("repeats-50M-30x150-k55", 0.003)):
        seq, off, p = synth.make(name, scale)
        k = p["k"]
        res = ctx.count(seq, off, k, p["p"], p["n_bins"], 1, 2**32 - 1,
                        flags=kmc.FLAG_DEVICE_TABLE)
        lut = 4 if k == 28 else 3
        db = kmc.Db.build(ctx, res, lut, 4)
        ok_keys, ok_counts = oracle.count(seq, off, k)
        table = dict(zip(as_ints(ok_keys), (int(c) for c in ok_counts)))
        rng = np.random.default_rng(k)
        present = [int(v) for v in rng.choice(list(table), 20000, replace=False)]
        # half of them asked in the other orientation
        q = [revcomp_int(v, k) if i % 2 else v for i, v in enumerate(present)]
        absent = []
        while len(absent) < 5000:
            v = int(rng.integers(0, 2**62)) % (4 ** k) if k <= 31 else \
                (int(rng.integers(0, 2**62)) << 62 | int(rng.integers(0, 2**62))) % (4 ** k)
            if min(v, revcomp_int(v, k)) not in table:
                absent.append(v)
        q += absent
        dq = pack_queries(q, k)
        out = torch.zeros(len(q), dtype=torch.int32, device="cuda:0")
        db.query(dq, out)
        got = out.cpu().numpy().view(np.uint32)
        want = [table.get(min(v, revcomp_int(v, k)), 0) for v in q]
        assert [int(x) for x in got] == want
        # SetMinCount / SetMaxCount: counts outside [2, 5] read as absent
        db.query(dq, out, min_count=2, max_count=5)
        got = out.cpu().numpy().view(np.uint32)
        assert [int(x) for x in got] == [c if 2 <= c <= 5 else 0 for c in want]
        res.free()
        db.free()


@pytest.mark.parametrize("k,lut,cs", [(32, 0, 1), (21, 1, 3), (33, 1, 2), (64, 0, 4),
                                      (40, 4, 1)])
def test_db_query_suffix_widths(ctx, kmc, k, lut, cs):
    # suffixes of 5 to 16 bytes, records of odd lengths (every alignment of a
    # record in the buffer), including the last record: lookups of every
    # entry (both orientations) and of absent k-mers against the oracle
    import torch
    seq, off = synth.sample_reads(k, synth.random_reference(k + 1, 20_000), 4000, (80, 160),
                                  0.01, 0.0)
    res = ctx.count(seq, off, k, 7, 64, 1, 2**32 - 1, flags=kmc.FLAG_DEVICE_TABLE)
    db = kmc.Db.build(ctx, res, lut, cs)
    ok_keys, ok_counts = oracle.count(seq, off, k)
    cap = 2 ** (8 * cs) - 1
    table = dict(zip(as_ints(ok_keys), (min(int(c), cap) for c in ok_counts)))
    q = [revcomp_int(v, k) if i % 2 else v for i, v in enumerate(table)]
    rng = np.random.default_rng(k)
    while len(q) < len(table) + 3000:
        v = (int(rng.integers(0, 2**62)) << 62 | int(rng.integers(0, 2**62))) % (4 ** k)
        if min(v, revcomp_int(v, k)) not in table:
            q.append(v)
    dq = pack_queries(q, k)
    out = torch.zeros(len(q), dtype=torch.int32, device="cuda:0")
    db.query(dq, out)
    got = out.cpu().numpy().view(np.uint32)
    assert [int(x) for x in got] == [table.get(min(v, revcomp_int(v, k)), 0) for v in q]
    res.free()
    db.free()


def test_db_open_decode_roundtrip(ctx, kmc, tmp_path):
    import torch
    seq, off, p = synth.make("genome-5M-2Mx100", 0.01)
    res = ctx.count(seq, off, 28, 7, 512, 2, 10**9, keep_table=True)
    db = kmc.Db.build(ctx, res, 4, 4)
    path = str(tmp_path / "rt")
    db.write(path)
    db2 = kmc.Db.open(ctx, path)
    assert db2.info == db.info
    keys = torch.zeros(res.n, dtype=torch.int64, device="cuda:0")
    counts = torch.zeros(res.n, dtype=torch.int32, device="cuda:0")
    db2.decode(keys, counts)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), res.keys)
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), res.counts)
    # the opened database answers like the built one
    dq = pack_queries([int(v) for v in res.keys[::97]], 28)
    a = torch.zeros(dq.numel(), dtype=torch.int32, device="cuda:0")
    b = torch.zeros_like(a)
    db.query(dq, a)
    db2.query(dq, b)
    assert torch.equal(a, b) and bool((a > 0).all())
    res.free()
    db.free()
    db2.free()


def test_db_supplement_examples(ctx, kmc, tmp_path):
    # ATACGACAAATG with signature length 5: signature ACGAC = 97 selects map
    # entry 97; with lut = 4 its prefix ATAC = 49 selects the record range,
    # where the suffix GACAAATG is found.  The prefix array of the signature
    # starts at byte 4 + map[97] * 4^lut * 8 of .kmc_pre.
    reads = ["ATACGACAAATG", "ATACGACAAATGC", "GGATACGACAAATGTT"]
    seq, off = to_reads(reads)
    res = ctx.count(seq, off, 12, 5, 64, 1, 2**32 - 1, keep_table=True)
    db = kmc.Db.build(ctx, res, 4, 4)
    path = str(tmp_path / "ex")
    db.write(path)
    d = read_db(path)
    assert S.encode(S.signature("ATACGACAAATG", 5)) == 97
    arr = int(d["map"][97])
    start = 4 + arr * 4 ** 4 * 8
    lo = struct.unpack_from("<Q", d["raw_pre"], start + 49 * 8)[0]
    hi = struct.unpack_from("<Q", d["raw_pre"], start + 50 * 8)[0]
    suffixes = [bytes(d["recs"][r][:2]) for r in range(lo, hi)]
    gacaaatg = bytes([0b10000100, 0b00001110])  # GACA, AATG
    assert gacaaatg in suffixes
    assert lookup(d, S.encode("ATACGACAAATG"), 5) == 3
    res.free()
    db.free()
    # CCACAAAT packs as 0x51 0x03: a database of k-mers as read, no prefix
    seq, off = to_reads(["CCACAAAT"])
    res = ctx.count(seq, off, 8, 4, 4, 1, 2**32 - 1, flags=kmc.FLAG_NON_CANONICAL,
                    keep_table=True)
    db = kmc.Db.build(ctx, res, 0, 1)
    db.write(path)
    d = read_db(path)
    assert d["tmp"][0] == kmc.FLAG_NON_CANONICAL
    assert [bytes(r) for r in d["recs"]] == [bytes([0x51, 0x03, 0x01])]
    res.free()
    db.free()


def test_db_rejects_bad_shapes_and_files(ctx, kmc, tmp_path):
    seq, off = to_reads(["ACGTACGTACGTACGTACGTACGTACGTACGTACG"])
    res = ctx.count(seq, off, 28, 7, 16, 1, 2**32 - 1, keep_table=True)
    for lut, cs in ((3, 4), (4, 0), (4, 5)):  # 4 must divide k - lut; counter 1..4 bytes
        with pytest.raises(kmc.KmcError) as e:
            kmc.Db.build(ctx, res, lut, cs)
        assert e.value.status == kmc.KMC_ERR_INVALID_ARG
    db = kmc.Db.build(ctx, res, 4, 4)
    path = str(tmp_path / "bad")
    db.write(path)
    raw = open(path + ".kmc_pre", "rb").read()
    open(path + ".kmc_pre", "wb").write(raw[:-1])  # truncated: no end marker
    with pytest.raises(kmc.KmcError) as e:
        kmc.Db.open(ctx, path)
    assert e.value.status == kmc.KMC_ERR_INVALID_ARG
    assert not os.path.exists(str(tmp_path / "missing.kmc_pre"))
    with pytest.raises(kmc.KmcError):
        kmc.Db.open(ctx, str(tmp_path / "missing"))
    res.free()
    db.free()
