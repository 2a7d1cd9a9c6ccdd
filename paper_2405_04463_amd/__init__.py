"""Python binding of libirismpc.so (the C ABI in include/irismpc.h).

Argument marshalling only: every step of the protocol runs in the library's
HIP kernels.  Device buffers are passed as torch CUDA tensors (used for their
memory and streams) or raw integer addresses.  The library must have been
built (``python -m paper_2405_04463_amd.build``); if it is missing this
module raises at first use instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libirismpc.so")

IMC_OK, IMC_EINVAL, IMC_ESHAPE, IMC_ENOMEM, IMC_EDEVICE, IMC_ECORRUPT, IMC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
OPEN_U8_XOR, OPEN_U64_XOR, OPEN_U16_ADD, OPEN_U32_ADD = 0, 1, 2, 3
CODE_BITS, CODE_WORDS, MAX_ROT, ENTRY_BYTES = 12800, 200, 32, 102400
NOALLOC_MAX_ROWS = 512   # rows of one imc_dot_shares_rows_noalloc call

EXPORTS = [
    "imc_create", "imc_destroy", "imc_strerror", "imc_db_bytes", "imc_query_op_bytes", "imc_query_raw_bytes",
    "imc_or_tree_ws_bytes", "imc_share_db", "imc_share_query", "imc_dot_shares", "imc_reshare",
    "imc_compare_threshold", "imc_or_tree", "imc_open", "imc_append_db", "imc_dot_shares_rows",
    "imc_set_dot_tiles", "imc_galois_db_bytes", "imc_galois_query_op_bytes", "imc_galois_query_raw_bytes",
    "imc_galois_share_db", "imc_galois_share_query", "imc_galois_dot_shares", "imc_galois_dot_shares_rows",
    "imc_galois_append_db", "imc_mask_in_batch", "imc_or_bits", "imc_dot_shares_gather",
    "imc_galois_dot_shares_gather", "imc_compare_variant", "imc_rotate_masks", "imc_plain_ml", "imc_db32_bytes",
    "imc_query32_op_bytes", "imc_share32_db", "imc_share32_query", "imc_dot32_shares", "imc_reshare32",
    "imc_dot_shares_rows_noalloc", "imc_compare_msg_bytes", "imc_or_pairs", "imc_dot_shares_groups",
    "imc_galois_dot_shares_groups", "imc_reshare_queries", "imc_compare_threshold_queries",
    "imc_compare_threshold_msgs",
]

(DOT_TILES_AUTO, DOT_TILES_EXPANDED_256x128, DOT_TILES_EXPANDED_128x128, DOT_TILES_EXPANDED_SHALLOW, DOT_TILES_ROTATION,
 DOT_TILES_ROTATION_LDSCOPY, DOT_TILES_ROTATION_DIRECT) = (0, 1, 2, 3, 4, 6, 7)
DOT_PERSISTENT = 0x10
CMP_PLAIN_MASK, CMP_LIFT18, CMP_CONST32 = 1, 2, 3   # imc_compare_variant settings


class IMCError(RuntimeError):
    def __init__(self, status: int, call: str):
        self.status = status
        super().__init__(f"{call}: {status} ({_strerror(status)})")


class imc_params(ctypes.Structure):
    _fields_ = [
        ("code_bits", ctypes.c_uint32),
        ("thr_a", ctypes.c_uint32),
        ("max_rows", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("dealer_key", ctypes.c_uint8 * 32),
        ("party_key", (ctypes.c_uint8 * 32) * 3),
    ]


class imc_row(ctypes.Structure):
    _fields_ = [("query_index", ctypes.c_uint32), ("rot", ctypes.c_int32)]


class imc_ids(ctypes.Structure):
    _fields_ = [
        ("query_id_base", ctypes.c_uint64),
        ("first_entry_id", ctypes.c_uint64),
        ("r", ctypes.c_int32),
        ("rot", ctypes.c_int8 * MAX_ROT),
    ]


MAX_DOT_GROUPS = 8


class imc_dot_group(ctypes.Structure):
    _fields_ = [
        ("qop", ctypes.c_void_p),
        ("q", ctypes.c_uint64),
        ("r", ctypes.c_int32),
        ("rot", ctypes.c_int8 * MAX_ROT),
        ("code_dot", ctypes.c_void_p),
        ("mask_dot", ctypes.c_void_p),
    ]


_VP = ctypes.c_void_p
_P3 = _VP * 3
_lib = None


def lib():
    """Load libirismpc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_04463_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        sz = ctypes.c_size_t
        st = ctypes.c_int
        L.imc_create.argtypes = [ctypes.POINTER(imc_params), ctypes.c_int, ctypes.POINTER(_VP)]
        L.imc_destroy.argtypes = [_VP]
        L.imc_destroy.restype = None
        L.imc_strerror.argtypes = [st]
        L.imc_strerror.restype = ctypes.c_char_p
        for f in ("imc_db_bytes", "imc_query_op_bytes", "imc_query_raw_bytes", "imc_galois_db_bytes",
                  "imc_galois_query_op_bytes", "imc_galois_query_raw_bytes", "imc_db32_bytes", "imc_query32_op_bytes"):
            getattr(L, f).argtypes = [sz]
            getattr(L, f).restype = sz
        L.imc_or_tree_ws_bytes.argtypes = [sz, sz, sz]
        L.imc_or_tree_ws_bytes.restype = sz
        L.imc_share_db.argtypes = [_VP, _VP, _VP, sz, ctypes.c_uint64, _P3, sz, _VP]
        L.imc_share_query.argtypes = [_VP, _VP, _VP, sz, ctypes.c_uint64, _P3, _VP, _VP]
        L.imc_dot_shares.argtypes = [_VP, ctypes.c_int, _VP, sz, ctypes.POINTER(imc_ids), _VP, sz, sz, _VP, _VP, sz, _VP]
        L.imc_reshare.argtypes = [_VP, _P3, _VP, sz, sz, sz, ctypes.POINTER(imc_ids), _P3, _VP, _VP, _VP]
        L.imc_compare_threshold_msgs.argtypes = [_VP, _P3, sz, sz, sz, ctypes.POINTER(imc_ids), _VP, sz, _P3, sz, _VP]
        L.imc_compare_threshold.argtypes = [_VP, _P3, _P3, sz, sz, sz, ctypes.POINTER(imc_ids), _VP, sz, _P3, sz, _VP]
        L.imc_reshare_queries.argtypes = [_VP, _P3, _VP, sz, sz, sz, ctypes.POINTER(imc_ids), _VP, _P3, _P3, _VP, _VP]
        L.imc_compare_threshold_queries.argtypes = [_VP, _P3, _P3, sz, sz, sz, ctypes.POINTER(imc_ids), _VP, _VP, sz,
                                                    sz, _VP]
        L.imc_compare_msg_bytes.argtypes = [ctypes.c_int, sz, sz]
        L.imc_compare_msg_bytes.restype = sz
        L.imc_or_tree.argtypes = [_VP, _P3, sz, sz, sz, ctypes.POINTER(imc_ids), _VP, sz, _P3, _VP]
        L.imc_open.argtypes = [_VP, ctypes.c_int, _P3, sz, _VP, ctypes.c_int, _VP]
        L.imc_append_db.argtypes = [_VP, _P3, sz, _P3, sz, ctypes.c_uint64, _VP]
        L.imc_dot_shares_rows.argtypes = [_VP, ctypes.c_int, _VP, sz, _VP, sz, _VP, sz, ctypes.c_uint64, sz, _VP, _VP,
                                          sz, _VP]
        L.imc_set_dot_tiles.argtypes = [_VP, ctypes.c_uint32]
        L.imc_galois_share_db.argtypes = L.imc_share_db.argtypes
        L.imc_galois_share_query.argtypes = L.imc_share_query.argtypes
        L.imc_galois_dot_shares.argtypes = L.imc_dot_shares.argtypes
        L.imc_galois_dot_shares_rows.argtypes = L.imc_dot_shares_rows.argtypes
        L.imc_dot_shares_rows_noalloc.argtypes = L.imc_dot_shares_rows.argtypes
        L.imc_galois_append_db.argtypes = L.imc_append_db.argtypes
        L.imc_mask_in_batch.argtypes = [_VP, _P3, sz, sz, sz, sz, sz, _VP]
        L.imc_or_pairs.argtypes = [_VP, _P3, sz, ctypes.c_uint64, _P3, _VP]
        L.imc_dot_shares_gather.argtypes = [_VP, ctypes.c_int, _VP, _VP, sz, ctypes.POINTER(imc_ids), _VP, sz, sz, _VP,
                                            _VP, sz, _VP]
        L.imc_galois_dot_shares_gather.argtypes = L.imc_dot_shares_gather.argtypes
        L.imc_dot_shares_groups.argtypes = [_VP, ctypes.c_int, ctypes.POINTER(imc_dot_group), sz, _VP, sz,
                                            ctypes.c_uint64, sz, sz, _VP]
        L.imc_galois_dot_shares_groups.argtypes = L.imc_dot_shares_groups.argtypes
        L.imc_or_bits.argtypes = [_VP, _P3, _P3, sz, ctypes.c_uint64, _P3, _VP]
        L.imc_compare_variant.argtypes = [_VP, ctypes.c_int, _P3, ctypes.c_int, _VP, _VP, sz, sz, sz,
                                          ctypes.POINTER(imc_ids), _VP, sz, _P3, sz, _VP]
        L.imc_rotate_masks.argtypes = [_VP, _VP, sz, ctypes.POINTER(imc_ids), _VP, _VP]
        L.imc_plain_ml.argtypes = [_VP, _VP, sz, _VP, sz, _VP, sz, _VP]
        L.imc_share32_db.argtypes = [_VP, ctypes.c_int, _VP, _VP, sz, ctypes.c_uint64, _P3, sz, _VP]
        L.imc_share32_query.argtypes = [_VP, ctypes.c_int, _VP, _VP, sz, ctypes.c_uint64, _P3, _VP]
        L.imc_dot32_shares.argtypes = [_VP, ctypes.c_int, _VP, sz, ctypes.POINTER(imc_ids), _VP, sz, sz, _VP, sz, _VP]
        L.imc_reshare32.argtypes = [_VP, ctypes.c_int, _P3, sz, sz, sz, ctypes.POINTER(imc_ids), _P3, _P3, _VP]
        for f in EXPORTS:
            if f not in ("imc_destroy", "imc_strerror") and not f.endswith("_bytes"):
                getattr(L, f).restype = st
        _lib = L
    return _lib


def _strerror(s: int) -> str:
    try:
        return lib().imc_strerror(s).decode()
    except Exception:  # noqa: BLE001 - message only
        return "?"


def _check(status: int, call: str) -> int:
    if status != IMC_OK:
        raise IMCError(status, call)
    return status


def addr(t) -> int:
    """Device address of a tensor (or an int address passed through)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _p3(ts):
    return _P3(*[addr(t) for t in ts])   # None -> NULL


def _stream(stream) -> int | None:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


QUERY_ENTRY_WORDS = 6   # imc_query_entry: query_id, n, match[3], match_plane (u64 each)


def query_table(entries, out=None):
    """Pack imc_query_entry rows: entries = [(query_id, n, (match0, match1, match2), match_plane), ...]
    with match pointers as tensors, addresses or None (match_plane in u64 words).  Returns (or fills)
    an int64 tensor [q][6] on the host; the caller copies it to the device."""
    import torch

    t = out if out is not None else torch.empty(len(entries), QUERY_ENTRY_WORDS, dtype=torch.int64)
    vals = []
    for qid, n, m3, plane in entries:
        ptrs = [addr(m) or 0 for m in (m3 if m3 is not None else (None, None, None))]
        vals.append([qid, n] + [x - (1 << 64) if x >= (1 << 63) else x for x in ptrs] + [plane])
    if vals:
        t[:len(vals)] = torch.tensor(vals, dtype=torch.int64)
    return t


def make_ids(query_id_base: int, rot, first_entry_id: int = 0) -> imc_ids:
    ids = imc_ids()
    ids.query_id_base = query_id_base
    ids.first_entry_id = first_entry_id
    ids.r = len(rot)
    for i, s in enumerate(rot):
        ids.rot[i] = int(s)
    return ids


# ---- sizes -------------------------------------------------------------
def db_bytes(capacity: int) -> int:
    return lib().imc_db_bytes(capacity)


def query_op_bytes(q: int) -> int:
    return lib().imc_query_op_bytes(q)


def query_raw_bytes(q: int) -> int:
    return lib().imc_query_raw_bytes(q)


def galois_db_bytes(capacity: int) -> int:
    return lib().imc_galois_db_bytes(capacity)


def galois_query_op_bytes(q: int) -> int:
    return lib().imc_galois_query_op_bytes(q)


def galois_query_raw_bytes(q: int) -> int:
    return lib().imc_galois_query_raw_bytes(q)


def db32_bytes(capacity: int) -> int:
    return lib().imc_db32_bytes(capacity)


def query32_op_bytes(q: int) -> int:
    return lib().imc_query32_op_bytes(q)


def or_tree_ws_bytes(q: int, r: int, nw: int) -> int:
    return lib().imc_or_tree_ws_bytes(q, r, nw)


def compare_msg_bytes(variant: int, rows: int, n: int) -> int:
    """Bytes of a comparison call's message buffer (variant 0 = MPCLift)."""
    return lib().imc_compare_msg_bytes(variant, rows, n)


@dataclass
class Keys:
    dealer: bytes
    party: bytes   # 3 x 32 bytes


class Context:
    """An imc_ctx on one device; methods mirror the C calls one to one."""

    def __init__(self, keys: Keys, max_rows: int, device: int = 0, dot_tiles: int = 0):
        p = imc_params()
        p.code_bits = CODE_BITS
        p.thr_a = 16384
        p.max_rows = max_rows
        p.flags = dot_tiles
        assert len(keys.dealer) == 32 and len(keys.party) == 96
        for i in range(32):
            p.dealer_key[i] = keys.dealer[i]
        for k in range(3):
            for i in range(32):
                p.party_key[k][i] = keys.party[32 * k + i]
        h = _VP()
        _check(lib().imc_create(ctypes.byref(p), device, ctypes.byref(h)), "imc_create")
        self._h = h
        self.device = device
        self.max_rows = max_rows

    def close(self):
        if getattr(self, "_h", None):
            lib().imc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    # -- imc_share_db / imc_galois_share_db
    def share_db(self, codes, masks, n, first_entry_id, db3, capacity, stream=None, galois=False):
        f = "imc_galois_share_db" if galois else "imc_share_db"
        return _check(getattr(lib(), f)(self._h, addr(codes), addr(masks), n, first_entry_id, _p3(db3), capacity,
                                        _stream(stream)), f)

    # -- imc_share_query / imc_galois_share_query
    def share_query(self, codes, masks, q, query_id_base, qop3, qraw3=None, stream=None, galois=False):
        f = "imc_galois_share_query" if galois else "imc_share_query"
        raw = _p3(qraw3) if qraw3 is not None else None
        return _check(getattr(lib(), f)(self._h, addr(codes), addr(masks), q, query_id_base, _p3(qop3),
                                        ctypes.cast(raw, _VP) if raw is not None else None, _stream(stream)), f)

    # -- imc_dot_shares / imc_galois_dot_shares
    def dot_shares(self, party, qop, q, ids: imc_ids, db, capacity, n, code_dot, mask_dot, ld, stream=None,
                   galois=False):
        f = "imc_galois_dot_shares" if galois else "imc_dot_shares"
        return _check(getattr(lib(), f)(self._h, party, addr(qop), q, ctypes.byref(ids), addr(db), capacity, n,
                                        addr(code_dot), addr(mask_dot), ld, _stream(stream)), f)

    # -- imc_dot_shares_gather / imc_galois_dot_shares_gather (qidx: device uint32/int32 tensor [q])
    def dot_shares_gather(self, party, qop, qidx, q, ids: imc_ids, db, capacity, n, code_dot, mask_dot, ld,
                          stream=None, galois=False):
        f = "imc_galois_dot_shares_gather" if galois else "imc_dot_shares_gather"
        return _check(getattr(lib(), f)(self._h, party, addr(qop), addr(qidx), q, ctypes.byref(ids), addr(db),
                                        capacity, n, addr(code_dot), addr(mask_dot), ld, _stream(stream)), f)

    # -- imc_dot_shares_groups / imc_galois_dot_shares_groups
    #    (groups: list of (qop, q, rot, code_dot, mask_dot), one fused launch)
    def dot_shares_groups(self, party, groups, db, capacity, first_entry_id, n, ld, stream=None, galois=False):
        arr = (imc_dot_group * max(1, len(groups)))()
        for g, (qop, q, rot, code_dot, mask_dot) in zip(arr, groups):
            g.qop, g.q, g.r = addr(qop), q, len(rot)
            for i, v in enumerate(rot):
                g.rot[i] = int(v)
            g.code_dot, g.mask_dot = addr(code_dot), addr(mask_dot)
        f = "imc_galois_dot_shares_groups" if galois else "imc_dot_shares_groups"
        return _check(getattr(lib(), f)(self._h, party, arr, len(groups), addr(db), capacity, first_entry_id, n, ld,
                                        _stream(stream)), f)

    # -- imc_dot_shares_rows / imc_galois_dot_shares_rows
    #    (rows: device int32 tensor [nrows, 2] = (query_index, rot))
    def dot_shares_rows(self, party, qop, q, rows, nrows, db, capacity, first_entry_id, n, code_dot, mask_dot, ld,
                        stream=None, galois=False):
        f = "imc_galois_dot_shares_rows" if galois else "imc_dot_shares_rows"
        return _check(getattr(lib(), f)(self._h, party, addr(qop), q, addr(rows), nrows, addr(db), capacity,
                                        first_entry_id, n, addr(code_dot), addr(mask_dot), ld, _stream(stream)), f)

    # -- imc_dot_shares_rows_noalloc (expanded rows in the library's static device array)
    def dot_shares_rows_noalloc(self, party, qop, q, rows, nrows, db, capacity, first_entry_id, n, code_dot, mask_dot,
                                ld, stream=None):
        return _check(lib().imc_dot_shares_rows_noalloc(self._h, party, addr(qop), q, addr(rows), nrows, addr(db),
                                                        capacity, first_entry_id, n, addr(code_dot), addr(mask_dot),
                                                        ld, _stream(stream)), "imc_dot_shares_rows_noalloc")

    # -- imc_set_dot_tiles
    def set_dot_tiles(self, flags: int):
        return _check(lib().imc_set_dot_tiles(self._h, flags), "imc_set_dot_tiles")

    # -- imc_reshare (add_mask3 / rep_mask3 None: code shares only; rep_code3 None: the messages only)
    def reshare(self, add_code3, add_mask3, rows, n, ld, ids: imc_ids, msg3, rep_code3, rep_mask3, stream=None):
        am = ctypes.cast(_p3(add_mask3), _VP) if add_mask3 is not None else None
        rc = ctypes.cast(_p3(rep_code3), _VP) if rep_code3 is not None else None
        rm = ctypes.cast(_p3(rep_mask3), _VP) if rep_mask3 is not None else None
        return _check(lib().imc_reshare(self._h, _p3(add_code3), am, rows, n, ld, ctypes.byref(ids),
                                        _p3(msg3), rc, rm, _stream(stream)), "imc_reshare")

    # -- imc_compare_threshold_msgs: the components read in place from the resharing's messages
    def compare_threshold_msgs(self, msg3, rows, n, ld, ids: imc_ids, match3, mw_ld, stream=None, msg_ws=None):
        mb = msg_ws.numel() * msg_ws.element_size() if msg_ws is not None else 0
        return _check(lib().imc_compare_threshold_msgs(self._h, _p3(msg3), rows, n, ld, ctypes.byref(ids),
                                                       addr(msg_ws), mb, _p3(match3), mw_ld, _stream(stream)),
                      "imc_compare_threshold_msgs")

    # -- imc_compare_variant (variant CMP_*; rep_mask3 None for CMP_PLAIN_MASK; msg_ws: message buffer
    #    of compare_msg_bytes(variant, rows, n) bytes, None: messages held in registers)
    def compare_variant(self, variant, rep_code3, code_bits, rep_mask3, ml_pub, rows, n, ld, ids: imc_ids, match3,
                        mw_ld, stream=None, msg_ws=None):
        rm = ctypes.cast(_p3(rep_mask3), _VP) if rep_mask3 is not None else None
        mb = msg_ws.numel() * msg_ws.element_size() if msg_ws is not None else 0
        return _check(lib().imc_compare_variant(self._h, variant, _p3(rep_code3), code_bits, rm, addr(ml_pub), rows,
                                                n, ld, ctypes.byref(ids), addr(msg_ws), mb, _p3(match3), mw_ld,
                                                _stream(stream)), "imc_compare_variant")

    # -- Z_2^32 sharing, dot products and resharing of one vector (vec 0 code, 1 mask)
    def share32_db(self, vec, codes, masks, n, first_entry_id, db3, capacity, stream=None):
        return _check(lib().imc_share32_db(self._h, vec, addr(codes), addr(masks), n, first_entry_id, _p3(db3),
                                           capacity, _stream(stream)), "imc_share32_db")

    def share32_query(self, vec, codes, masks, q, query_id_base, qop3, stream=None):
        return _check(lib().imc_share32_query(self._h, vec, addr(codes), addr(masks), q, query_id_base, _p3(qop3),
                                              _stream(stream)), "imc_share32_query")

    def dot32_shares(self, party, qop, q, ids: imc_ids, db, capacity, n, dot, ld, stream=None):
        return _check(lib().imc_dot32_shares(self._h, party, addr(qop), q, ctypes.byref(ids), addr(db), capacity, n,
                                             addr(dot), ld, _stream(stream)), "imc_dot32_shares")

    def reshare32(self, vec, add3, rows, n, ld, ids: imc_ids, msg3, rep3, stream=None):
        return _check(lib().imc_reshare32(self._h, vec, _p3(add3), rows, n, ld, ctypes.byref(ids), _p3(msg3),
                                          _p3(rep3), _stream(stream)), "imc_reshare32")

    # -- imc_rotate_masks / imc_plain_ml (masks in plain)
    def rotate_masks(self, masks, q, ids: imc_ids, out, stream=None):
        return _check(lib().imc_rotate_masks(self._h, addr(masks), q, ctypes.byref(ids), addr(out), _stream(stream)),
                      "imc_rotate_masks")

    def plain_ml(self, row_masks, rows, db_masks, n, ml, ld, stream=None):
        return _check(lib().imc_plain_ml(self._h, addr(row_masks), rows, addr(db_masks), n, addr(ml), ld,
                                         _stream(stream)), "imc_plain_ml")

    # -- imc_compare_threshold (msg_ws: device tensor of compare_msg_bytes(0, rows, n) bytes, the
    #    message buffer between the parties; None: messages held in registers)
    def compare_threshold(self, rep_code3, rep_mask3, rows, n, ld, ids: imc_ids, match3, mw_ld, stream=None,
                          msg_ws=None):
        mb = msg_ws.numel() * msg_ws.element_size() if msg_ws is not None else 0
        return _check(lib().imc_compare_threshold(self._h, _p3(rep_code3), _p3(rep_mask3), rows, n, ld,
                                                  ctypes.byref(ids), addr(msg_ws), mb, _p3(match3), mw_ld,
                                                  _stream(stream)), "imc_compare_threshold")

    # -- imc_reshare_queries / imc_compare_threshold_queries: the rows of q queries that each carry
    #    their own id, column count and match buffer (table: device tensor of q imc_query_entry rows,
    #    see query_table)
    def reshare_queries(self, add_code3, add_mask3, q, n, ld, ids: imc_ids, table, msg3, rep_code3, rep_mask3,
                        stream=None):
        am = ctypes.cast(_p3(add_mask3), _VP) if add_mask3 is not None else None
        rm = ctypes.cast(_p3(rep_mask3), _VP) if rep_mask3 is not None else None
        return _check(lib().imc_reshare_queries(self._h, _p3(add_code3), am, q, n, ld, ctypes.byref(ids), addr(table),
                                                _p3(msg3), _p3(rep_code3), rm, _stream(stream)),
                      "imc_reshare_queries")

    def compare_threshold_queries(self, rep_code3, rep_mask3, q, n, ld, ids: imc_ids, table, mw_ld, stream=None,
                                  msg_ws=None):
        mb = msg_ws.numel() * msg_ws.element_size() if msg_ws is not None else 0
        return _check(lib().imc_compare_threshold_queries(self._h, _p3(rep_code3), _p3(rep_mask3), q, n, ld,
                                                          ctypes.byref(ids), addr(table), addr(msg_ws), mb, mw_ld,
                                                          _stream(stream)), "imc_compare_threshold_queries")

    # -- imc_or_tree
    def or_tree(self, match3, q, nw, mw_ld, ids: imc_ids, ws, ws_bytes, dup3, stream=None):
        return _check(lib().imc_or_tree(self._h, _p3(match3), q, nw, mw_ld, ctypes.byref(ids), addr(ws), ws_bytes,
                                        _p3(dup3), _stream(stream)), "imc_or_tree")

    # -- imc_mask_in_batch (group: consecutive queries that may not match each other, e.g. 2 eyes)
    def mask_in_batch(self, match3, q, r, mw_ld, word, stream=None, group=1):
        return _check(lib().imc_mask_in_batch(self._h, _p3(match3), q, r, mw_ld, word, group, _stream(stream)),
                      "imc_mask_in_batch")

    # -- imc_or_pairs (element i of out = elements 2i OR 2i+1 of in)
    def or_pairs(self, in3, count, id_, out3, stream=None):
        return _check(lib().imc_or_pairs(self._h, _p3(in3), count, id_, _p3(out3), _stream(stream)), "imc_or_pairs")

    # -- imc_or_bits
    def or_bits(self, a3, b3, count, id_, out3, stream=None):
        return _check(lib().imc_or_bits(self._h, _p3(a3), _p3(b3), count, id_, _p3(out3), _stream(stream)),
                      "imc_or_bits")

    # -- imc_open (returns the status: IMC_ECORRUPT is reported, not raised)
    def open(self, kind, rep3, count, out, check=0, stream=None):
        s = lib().imc_open(self._h, kind, _p3(rep3), count, addr(out), int(check), _stream(stream))
        if s not in (IMC_OK, IMC_ECORRUPT):
            raise IMCError(s, "imc_open")
        return s

    # -- imc_append_db / imc_galois_append_db
    def append_db(self, qraw3, qi, db3, capacity, entry_id, stream=None, galois=False):
        f = "imc_galois_append_db" if galois else "imc_append_db"
        return _check(getattr(lib(), f)(self._h, _p3(qraw3), qi, _p3(db3), capacity, entry_id, _stream(stream)), f)
