"""Seeded synthetic workloads for the iris uniqueness check.

This module only generates inputs (packed iris codes and masks, planted
near-duplicate queries).  It holds none of the protocol's arithmetic and is
the one piece of code that both the CPU oracle's tests and the GPU path use.

Bit layout: a code has 12,800 bits, bit ``i`` sits in u64 word ``i >> 6`` at
bit ``i & 63``; ``i = ((row*200 + col)*2 + f)*2 + j`` with 16 angular rows of
200 columns.  A rotation by ``s`` moves column ``col`` to ``col + s`` (mod 200)
inside each row, for code and mask alike.

Bulk entries come from ``gen.c`` (SplitMix64 at a counter, so any entry can be
regenerated from its id).  Planted queries copy a database entry's code under
a fresh mask and flip an exact number of bits inside the combined mask at a
chosen rotation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

L = 12800
WORDS = 200
ROWS, COLS = 16, 200

CLS_DB_CODE, CLS_DB_MASK, CLS_Q_CODE, CLS_Q_MASK = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libwlgen.so")
_lib = None


def build_lib() -> str:
    """Compile the generator (gcc, OpenMP)."""
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB, os.path.join(_HERE, "gen.c")]
    )
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        lib = ctypes.CDLL(_LIB)
        lib.wl_codes.argtypes = [ctypes.c_uint64] * 4 + [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
        lib.wl_codes.restype = None
        lib.wl_word.argtypes = [ctypes.c_uint64] * 4
        lib.wl_word.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def gen_codes(seed: int, first: int, n: int, query: bool = False, out=None):
    """Codes and masks of ids ``first..first+n-1`` as two uint64 [n, 200] arrays."""
    lib = _load()
    if out is None:
        codes = np.empty((n, WORDS), dtype=np.uint64)
        masks = np.empty((n, WORDS), dtype=np.uint64)
    else:
        codes, masks = out
        assert codes.shape == (n, WORDS) and masks.shape == (n, WORDS)
        assert codes.flags.c_contiguous and masks.flags.c_contiguous
    cc, cm = (CLS_Q_CODE, CLS_Q_MASK) if query else (CLS_DB_CODE, CLS_DB_MASK)
    if n:
        lib.wl_codes(seed, cc, cm, first, n, codes.ctypes.data, masks.ctypes.data)
    return codes, masks


# --------------------------------------------------------------------------
# bit helpers (numpy, for planting only)
# --------------------------------------------------------------------------
def unpack(words: np.ndarray) -> np.ndarray:
    """uint64 [..., 200] -> uint8 bits [..., 12800] (bit i of the code)."""
    w = np.ascontiguousarray(words, dtype="<u8")
    b = np.unpackbits(w.view(np.uint8), axis=-1, bitorder="little")
    return b


def pack(bits: np.ndarray) -> np.ndarray:
    """uint8 bits [..., 12800] -> uint64 [..., 200]."""
    b = np.packbits(np.ascontiguousarray(bits, dtype=np.uint8), axis=-1, bitorder="little")
    return b.view("<u8").astype(np.uint64)


def rotate_bits(bits: np.ndarray, s: int) -> np.ndarray:
    """rot_s(v)[row][col][.] = v[row][(col - s) mod 200][.] on unpacked bits."""
    v = bits.reshape(bits.shape[:-1] + (ROWS, COLS, 4))
    return np.roll(v, s, axis=-2).reshape(bits.shape)


def _rng(seed: int, tag: int, qid: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed & (2**63 - 1), tag, qid])))


def plant(seed: int, qid: int, entry_code: np.ndarray, entry_mask: np.ndarray, s: int,
          h: float | None = None, exact: str | None = None):
    """A query that, at rotation ``s``, is a near-duplicate of the given entry.

    The query mask is a fresh Bernoulli(0.9) draw (this query's own mask
    stream, in the rotated frame); with ``ml`` the size of the combined mask,
    exactly ``floor(h*ml + 1/2)`` code bits inside it are flipped.
    ``exact='eq'`` makes 8*hd == 3*ml (not a match), ``exact='lt'`` makes
    8*hd == 3*ml - 1 (a match), by clearing the lowest combined-mask bits of
    the query mask until ``ml`` has the needed residue mod 8.
    Returns packed (code, mask) in the query's unrotated frame.
    """
    _, qm = gen_codes(seed, qid, 1, query=True)
    mt = unpack(qm[0])
    C = unpack(entry_code)
    M = unpack(entry_mask)
    comb = mt & M
    ml = int(comb.sum())
    if exact is not None:
        want = 0 if exact == "eq" else 3
        pos = np.flatnonzero(comb)
        k = 0
        while (ml - k) % 8 != want:
            k += 1
        mt = mt.copy()
        mt[pos[:k]] = 0
        comb = mt & M
        ml = int(comb.sum())
        flips = (3 * ml) // 8 if exact == "eq" else (3 * ml - 1) // 8
    else:
        flips = int(np.floor(h * ml + 0.5))
    pos = np.flatnonzero(comb)
    sel = _rng(seed, 7, qid).permutation(pos)[:flips]
    ct = C.copy()
    ct[sel] ^= 1
    return pack(rotate_bits(ct, -s)), pack(rotate_bits(mt, -s))


# --------------------------------------------------------------------------
# workload recipes (sizes and distributions of the paper-scale runs)
# --------------------------------------------------------------------------
ROT31 = list(range(-15, 16))


def rotations(r: int) -> list[int]:
    """Centred rotation offsets: 1 -> [0], 15 -> [-7..7], 31 -> [-15..15]."""
    h = (r - 1) // 2
    return list(range(-h, h + 1))


@dataclass
class Workload:
    name: str
    n_db: int
    n_q: int
    rot: list
    seed: int
    planted: list = field(default_factory=list)   # (query idx, entry, rot, h or exact)
    batch_pairs: list = field(default_factory=list)   # (query i, query j, rot, h or exact): i from j
    group: int = 1                                # queries per person (2: left and right eye)

    @property
    def rows(self) -> int:
        return self.n_q * len(self.rot)


def small_plain(seed: int = 0x1A150001) -> Workload:
    """1,000 entries, 16 queries, no rotation, 4 planted at HD 0.20."""
    w = Workload("db1000_q16_r1", 1000, 16, [0], seed)
    rng = _rng(seed, 1, 0)
    ents = rng.choice(1000, size=4, replace=False)
    for qi, e in zip((1, 5, 9, 13), ents):
        w.planted.append((qi, int(e), 0, 0.20))
    return w


def full_protocol(n_db: int = 300_000, n_q: int = 64, seed: int = 0x1A150003) -> Workload:
    """3-party full protocol: n_db entries, n_q queries x 31 rotations; half the
    queries planted with HD ~ U[0.15, 0.45] at a random entry and rotation, plus
    two exact-threshold and two threshold-minus-one cases."""
    w = Workload(f"db{n_db}_q{n_q}_r31", n_db, n_q, ROT31, seed)
    rng = _rng(seed, 3, 0)
    nplant = n_q // 2
    for qi in range(nplant):
        e = int(rng.integers(0, n_db))
        s = int(rng.integers(-15, 16))
        w.planted.append((2 * qi, e, s, float(rng.uniform(0.15, 0.45))))
    extra = [(2 * i + 1, ex) for i, ex in zip(range(min(4, n_q // 2)), ("eq", "lt", "eq", "lt"))]
    for qi, ex in extra:
        e = int(rng.integers(0, n_db))
        s = int(rng.integers(-15, 16))
        w.planted.append((qi, e, s, ex))
    return w


def party_local(n_db: int = 1_000_000, n_q: int = 32, seed: int = 0x1A150002) -> Workload:
    """One party's dot products: n_db entries vs n_q queries x 31 rotations."""
    w = Workload(f"db{n_db}_q{n_q}_r31", n_db, n_q, ROT31, seed)
    rng = _rng(seed, 2, 0)
    for qi in range(n_q):
        e = int(rng.integers(0, n_db))
        s = int(rng.integers(-15, 16))
        w.planted.append((qi, e, s, 0.20))
    return w


def two_eyes(n_db: int = 300_000, persons: int = 32, seed: int = 0x1A150005) -> Workload:
    """A batch of persons, each a query of both eyes (query 2k: left eye of
    person k, 2k+1: right eye) x 31 rotations, with the patterns a person
    decision has to get right.  Persons k = 4i: left eye planted against the
    database (HD ~ U[0.15, 0.45]); 4i+1: right eye; 4i+2: both eyes (two
    entries); 4i+3: neither, except person 3 (left eye exactly at the
    threshold: no match) and person 7 (right eye one below: a match).
    In-batch pairs (eye i made from eye j): a later person's eye from an
    earlier person's (counts), an eye from a later person's (counts for the
    later person only), a right eye from the same person's left eye (never
    counts: a person's eyes are not matched with each other), and two
    exact-threshold cases."""
    n_q = 2 * persons
    w = Workload(f"db{n_db}_persons{persons}_eyes2_r31", n_db, n_q, ROT31, seed, group=2)
    rng = _rng(seed, 5, 0)

    def entry():
        return int(rng.integers(0, n_db)), int(rng.integers(-15, 16))

    for k in range(persons):
        eyes = {0: (0,), 1: (1,), 2: (0, 1), 3: ()}[k % 4]
        for eye in eyes:
            e, s = entry()
            w.planted.append((2 * k + eye, e, s, float(rng.uniform(0.15, 0.45))))
    for k, eye, ex in ((3, 0, "eq"), (7, 1, "lt")):
        if k < persons:
            e, s = entry()
            w.planted.append((2 * k + eye, e, s, ex))
    pairs = ((22, 6, 3, 0.20),      # person 11 left from person 3 left (earlier person)
             (31, 30, 0, 0.10),     # person 15 right from its own left eye (not a duplicate)
             (46, 55, -6, 0.25),    # person 23 left from person 27 right (counts for person 27)
             (39, 14, -4, "lt"),    # person 19 right from person 7 left, one below the threshold
             (62, 23, 9, "eq"))     # person 31 left from person 11 right, exactly at the threshold
    w.batch_pairs = [p for p in pairs if max(p[0], p[1]) < n_q]
    return w


def plant_in_batch(w: Workload, qc: np.ndarray, qm: np.ndarray,
                   pairs=((9, 4, 3, 0.20), (11, 2, -5, 0.30), (13, 12, 0, 0.42), (15, 14, 7, "eq"))):
    """Make query i of the batch a near-duplicate of query j (at rotation s,
    with fractional HD h or an exact-threshold case): the duplicates that
    only in-batch matching finds (for i if j is earlier, else for j).
    Modifies qc, qm in place."""
    for i, j, s, hx in pairs:
        assert i != j and max(i, j) < qc.shape[0]
        if isinstance(hx, str):
            c, m = plant(w.seed, i, qc[j], qm[j], s, exact=hx)
        else:
            c, m = plant(w.seed, i, qc[j], qm[j], s, h=hx)
        qc[i], qm[i] = c, m
    return qc, qm


def make_queries(w: Workload, db_lookup=None):
    """Packed (codes, masks) [n_q, 200] for a workload.  ``db_lookup(e)``
    returns the packed (code, mask) of entry e (default: regenerate it)."""
    qc, qm = gen_codes(w.seed, 0, w.n_q, query=True)
    for qi, e, s, hx in w.planted:
        if db_lookup is None:
            ec, em = gen_codes(w.seed, e, 1)
            ec, em = ec[0], em[0]
        else:
            ec, em = db_lookup(e)
        if isinstance(hx, str):
            c, m = plant(w.seed, qi, ec, em, s, exact=hx)
        else:
            c, m = plant(w.seed, qi, ec, em, s, h=hx)
        qc[qi], qm[qi] = c, m
    return qc, qm
