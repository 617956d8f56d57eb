"""Generic bitplane encoding of integer coefficient streams (Section V-C;
Section VI-C "optimized generic bitplane encoding"; Table I "generic
bitplane").

Sign-magnitude planes, most significant plane first.  A value's sign is
recorded in the plane where its first 1-bit appears, so planes above a
value's leading bit cost it nothing but its magnitude bit.  The paper gives no
byte layout; the one used here (shared with the GPU path only through this
written description) is:

  n   = number of codes, B = bit length of max |q| (0 for an all-zero stream)
  M   = ceil(n / 64) magnitude words per plane, C = ceil(n / 4096) chunks
  plane j = 0 .. B-1 holds bit b = B-1-j.

  index section  B*C little-endian uint32, plane-major: entry (j, c) = number
                 of codes whose leading bit is b among codes [0, 4096*c)
                 (lets a decoder place sign bits chunk by chunk); zero padded
                 to a multiple of 8 bytes
  magnitude      B*M little-endian uint64, plane-major: bit i of word w is
                 bit b of |q[64*w + i]| (zero beyond n)
  sign           plane-major, ceil(nsig_j / 64) uint64 words per plane: one
                 bit per code whose leading bit is b, in stream order, least
                 significant bit first, 1 = negative

Fetching the first k planes reads k*C index entries, k*M magnitude words and
the first k sign segments: bytes_j = 4*C + 8*M + 8*ceil(nsig_j / 64) per plane.

Lossless stage (Section V: the coefficients are stored with bitplane
encoding followed by lossless compression; the paper does not name the
lossless coder).  Reading: zero-word suppression of each plane's magnitude
words.  With nnz_j the plane's nonzero magnitude words, the plane is stored
suppressed when 8*C + 8*ceil(C/2) + 8*nnz_j < 8*M, else raw; a suppressed
plane is C uint64 presence words (bit i of word c set when word 64*c + i is
nonzero), C uint32 counts of nonzero words before chunk c (zero padded to 8
bytes), then its nonzero words in order.  A lossless blob is the index
section, every plane's magnitude section (raw or suppressed) in plane order,
then the sign section; bytes_j uses the plane's stored magnitude size.
Decoding k planes yields |q| with its low B-k bits cleared (truncation toward
zero), so the error left by a stream after k planes is
  delta(0) = max |q|,  delta(k) = 2**(B-k) - 1  (1 <= k <= B).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

CHUNK = 4096


@dataclass
class StreamMeta:
    n: int
    B: int
    maxabs: int
    nsig: List[int] = field(default_factory=list)
    lossless: bool = False
    nnz: List[int] = field(default_factory=list)   # nonzero magnitude words per plane
    encoding: str = "generic"   # "generic", "negabinary" or "negabinary_xor"

    @property
    def words(self) -> int:
        return (self.n + 63) // 64

    @property
    def chunks(self) -> int:
        return (self.n + CHUNK - 1) // CHUNK

    def suppressed(self, j: int) -> bool:
        C = self.chunks
        return self.lossless and 8 * C + 8 * ((C + 1) // 2) + 8 * self.nnz[j] < 8 * self.words

    def mag_bytes(self, j: int) -> int:
        """Stored bytes of plane j's magnitude words."""
        if self.suppressed(j):
            C = self.chunks
            return 8 * C + 8 * ((C + 1) // 2) + 8 * self.nnz[j]
        return 8 * self.words

    @property
    def negabinary(self) -> bool:
        return self.encoding != "generic"

    def plane_bytes(self, j: int) -> int:
        if self.negabinary:  # digit planes only: no index, no signs
            return self.mag_bytes(j)
        return 4 * self.chunks + self.mag_bytes(j) + 8 * ((self.nsig[j] + 63) // 64)

    def delta(self, k: int) -> int:
        if k <= 0:
            return self.maxabs
        if self.negabinary:
            return nb_delta(self.B, k)
        return (1 << (self.B - k)) - 1


# ---------------------------------------------------------------------------
# Negabinary encoding (Table I, PSNR mode: "negabinary with XOR").  A code q
# is written in base -2 with B digits, w = (q + A) ^ A where A has the odd
# bit positions set; digit planes are stored most significant first, with no
# sign bits.  B is the fewest digits whose range [-2(4^floor(B/2) - 1)/3,
# (4^ceil(B/2) - 1)/3] holds [-maxabs, maxabs].  Truncating to the first k
# planes keeps the top k digits (the rest set to 0); the dropped digits are
# worth between -2(4^floor(r/2) - 1)/3 and (4^ceil(r/2) - 1)/3 with r = B - k,
# so the error is at most floor((2^(r+1) - 1) / 3) (0 planes: maxabs).
# Reading of "XOR" (the paper gives no definition): every stored digit plane
# after the first is the XOR of the digit plane with the one above it, which
# the decoder undoes from the planes it has already read.
# ---------------------------------------------------------------------------

def nb_digits(V: int) -> int:
    n = 0
    while (4 ** ((n + 1) // 2) - 1) // 3 < V or 2 * (4 ** (n // 2) - 1) // 3 < V:
        n += 1
    return n


def nb_delta(B: int, k: int) -> int:
    r = B - k
    return (2 ** (r + 1) - 1) // 3


def nb_mask(B: int) -> int:
    return sum(1 << i for i in range(1, B, 2))


def to_negabinary(q: np.ndarray, B: int) -> np.ndarray:
    A = np.int64(nb_mask(B))
    return (np.asarray(q, dtype=np.int64) + A) ^ A


def from_negabinary(w: np.ndarray, B: int) -> np.ndarray:
    A = np.int64(nb_mask(B))
    return (np.asarray(w, dtype=np.int64) ^ A) - A


def truncate_nb(q: np.ndarray, B: int, k: int) -> np.ndarray:
    """What decoding the first k digit planes returns."""
    k = max(0, min(int(k), B))
    w = to_negabinary(q, B)
    keep = np.int64(((1 << B) - 1) & ~((1 << (B - k)) - 1))
    return from_negabinary(w & keep, B)


def encode_nb(q: np.ndarray, xor: bool, lossless: bool = False):
    """Negabinary digit planes (XOR-chained with ``xor``); returns (blob,
    StreamMeta).  Blob = the stored digit planes in order (raw, or zero-word
    suppressed with ``lossless``)."""
    q = np.asarray(q, dtype=np.int64).ravel()
    n = q.size
    maxabs = int(np.abs(q).max()) if n else 0
    B = nb_digits(maxabs)
    meta = StreamMeta(n=n, B=B, maxabs=maxabs, nsig=[0] * B, lossless=bool(lossless),
                      encoding="negabinary_xor" if xor else "negabinary")
    M, C = meta.words, meta.chunks
    w = to_negabinary(q, B)
    planes, prev = [], None
    for j in range(B):
        bits = ((w >> (B - 1 - j)) & 1).astype(np.uint8)
        raw = np.frombuffer(_pack_bits(bits, M), dtype="<u8")
        stored = raw ^ prev if (xor and prev is not None) else raw
        prev = raw
        planes.append(stored.astype("<u8").tobytes())
    if lossless:
        for j in range(B):
            meta.nnz.append(int(np.count_nonzero(np.frombuffer(planes[j], dtype="<u8"))))
            if meta.suppressed(j):
                planes[j] = suppress_plane(planes[j], M, C)
    return b"".join(planes), meta


def decode_nb(blob: bytes, meta: StreamMeta, k: int) -> np.ndarray:
    n, B = meta.n, meta.B
    k = max(0, min(int(k), B))
    w = np.zeros(n, dtype=np.int64)
    prev = None
    for j in range(k):
        stored = np.frombuffer(plane_words(blob, meta, j), dtype="<u8")
        raw = stored ^ prev if (meta.encoding == "negabinary_xor" and prev is not None) else stored
        prev = raw
        bits = _unpack_bits(raw.astype("<u8").tobytes(), n)
        w |= bits << (B - 1 - j)
    return from_negabinary(w, B)


def bitlength(mag: np.ndarray) -> np.ndarray:
    """Bit length of each non-negative int64 (0 for 0), bit by bit."""
    out = np.zeros(mag.shape, dtype=np.int64)
    for b in range(63):
        out[((mag >> b) & 1) == 1] = b + 1
    return out


def _pack_bits(bits: np.ndarray, nwords: int) -> bytes:
    padded = np.zeros(nwords * 64, dtype=np.uint8)
    padded[: bits.size] = bits
    return np.packbits(padded, bitorder="little").tobytes()


def _unpack_bits(buf: bytes, nbits: int) -> np.ndarray:
    arr = np.frombuffer(buf, dtype=np.uint8)
    return np.unpackbits(arr, bitorder="little")[:nbits].astype(np.int64)


def suppress_plane(raw: bytes, M: int, C: int) -> bytes:
    """Zero-word suppressed form of one plane's M magnitude words."""
    words = np.frombuffer(raw, dtype="<u8")
    presence, counts, kept = [], [], []
    before = 0
    for c in range(C):
        bits = 0
        for i in range(64):
            w = 64 * c + i
            if w < M and int(words[w]) != 0:
                bits |= 1 << i
                kept.append(int(words[w]))
        presence.append(bits)
        counts.append(before)
        before += bin(bits).count("1")
    out = np.array(presence, dtype="<u8").tobytes()
    cnt = np.array(counts, dtype="<u4").tobytes()
    out += cnt + b"\0" * ((-len(cnt)) % 8)
    return out + np.array(kept, dtype="<u8").tobytes()


def expand_plane(sec: bytes, M: int, C: int) -> bytes:
    """Raw magnitude words of a suppressed plane (inverse of suppress_plane)."""
    presence = np.frombuffer(sec[: 8 * C], dtype="<u8")
    off = 8 * C + 8 * ((C + 1) // 2)
    kept = np.frombuffer(sec[off:], dtype="<u8")
    words = np.zeros(M, dtype="<u8")
    k = 0
    for c in range(C):
        bits = int(presence[c])
        for i in range(64):
            if (bits >> i) & 1:
                words[64 * c + i] = kept[k]
                k += 1
    return words.tobytes()


def encode(q: np.ndarray, lossless: bool = False):
    """Encode an int64 stream; returns (blob bytes, StreamMeta).  With
    ``lossless`` the magnitude planes are stored zero-word suppressed where
    that is smaller (see the module description)."""
    q = np.asarray(q, dtype=np.int64).ravel()
    n = q.size
    mag = np.abs(q)
    maxabs = int(mag.max()) if n else 0
    B = maxabs.bit_length()
    meta = StreamMeta(n=n, B=B, maxabs=maxabs, lossless=bool(lossless))
    M, C = meta.words, meta.chunks
    blen = bitlength(mag)
    index_parts, mag_parts, sign_parts = [], [], []
    for j in range(B):
        b = B - 1 - j
        bits = ((mag >> b) & 1).astype(np.uint8)
        mag_parts.append(_pack_bits(bits, M))
        newsig = blen == (b + 1)
        meta.nsig.append(int(newsig.sum()))
        signs = (q[newsig] < 0).astype(np.uint8)
        sign_parts.append(_pack_bits(signs, (signs.size + 63) // 64))
        before = np.concatenate([[0], np.cumsum(newsig.astype(np.int64))])
        idx = np.array([before[min(CHUNK * c, n)] for c in range(C)], dtype="<u4")
        index_parts.append(idx.tobytes())
    index = b"".join(index_parts)
    index += b"\0" * ((-len(index)) % 8)
    if lossless:
        for j in range(B):
            meta.nnz.append(int(np.count_nonzero(np.frombuffer(mag_parts[j], dtype="<u8"))))
            if meta.suppressed(j):
                mag_parts[j] = suppress_plane(mag_parts[j], M, C)
    blob = index + b"".join(mag_parts) + b"".join(sign_parts)
    return blob, meta


def section_offsets(meta: StreamMeta):
    """Byte offsets (index, magnitude, sign) of the three sections of a blob
    (a negabinary blob has only the plane section)."""
    if meta.negabinary:
        return 0, 0, sum(meta.mag_bytes(j) for j in range(meta.B))
    ib = 4 * meta.B * meta.chunks
    ib += (-ib) % 8
    return 0, ib, ib + sum(meta.mag_bytes(j) for j in range(meta.B))


def plane_words(blob: bytes, meta: StreamMeta, j: int) -> bytes:
    """Raw magnitude words of plane j (expanded if stored suppressed)."""
    _, moff, _ = section_offsets(meta)
    start = moff + sum(meta.mag_bytes(i) for i in range(j))
    sec = blob[start: start + meta.mag_bytes(j)]
    if meta.suppressed(j):
        return expand_plane(sec, meta.words, meta.chunks)
    return sec


def decode(blob: bytes, meta: StreamMeta, k: int) -> np.ndarray:
    """Decode the first k planes of a stream, reading magnitude and sign bits."""
    if meta.negabinary:
        return decode_nb(blob, meta, k)
    n, B = meta.n, meta.B
    k = max(0, min(int(k), B))
    mag = np.zeros(n, dtype=np.int64)
    neg = np.zeros(n, dtype=bool)
    _, moff, soff = section_offsets(meta)
    for j in range(k):
        b = B - 1 - j
        bits = _unpack_bits(plane_words(blob, meta, j), n)
        newsig = (mag == 0) & (bits == 1)
        nwords = (meta.nsig[j] + 63) // 64
        sbits = _unpack_bits(blob[soff: soff + 8 * nwords], meta.nsig[j])
        soff += 8 * nwords
        assert int(newsig.sum()) == meta.nsig[j]
        neg[newsig] = sbits == 1
        mag |= bits << b
    return np.where(neg, -mag, mag)


def read_index(blob: bytes, meta: StreamMeta) -> np.ndarray:
    """Index section as a (B, C) uint32 array."""
    C = meta.chunks
    raw = np.frombuffer(blob[: 4 * meta.B * C], dtype="<u4")
    return raw.reshape(meta.B, C) if meta.B else raw.reshape(0, C)


def truncate(q: np.ndarray, B: int, k: int) -> np.ndarray:
    """|q| with its low B-k bits cleared, sign kept (what decode(k) returns)."""
    q = np.asarray(q, dtype=np.int64)
    if k <= 0:
        return np.zeros_like(q)
    if k >= B:
        return q.copy()
    mask = ~np.int64((1 << (B - k)) - 1)
    mag = np.abs(q) & mask
    return np.where(q < 0, -mag, mag)
