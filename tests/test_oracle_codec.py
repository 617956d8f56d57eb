"""Pins of the coefficient decomposition (Section V-B) and the generic
bitplane codec (Section VI-C) against exact properties: round trips, the
norm-1 error lemma of integer lifting, zero residuals on even ramps, and a
bit-by-bit scalar re-implementation of the written byte layout."""
import itertools

import numpy as np
import pytest

from oracle import bitplane, cd


# ----------------------------------------------------------------- lifting

@pytest.mark.parametrize("shape,a", [((5, 9, 7), 0), ((5, 9, 7), 1), ((5, 9, 7), 2), ((4, 13), 0), ((4, 13), 1),
                                     ((1, 1, 6), 2), ((3, 1, 1), 0), ((0, 4, 4), 1), ((8, 8, 8), 0)])
def test_cd_round_trip(shape, a):
    rng = np.random.default_rng(1)
    R = rng.integers(-2**29, 2**29, size=shape)
    streams = cd.forward(R, a)
    assert sum(s.size for s in streams) == R.size
    np.testing.assert_array_equal(cd.inverse(streams, shape, a), R)


def test_cd_stream_order_is_lattice_row_major():
    """S1 lists the stride-4 points in the lattice's own row-major order."""
    shape = (3, 9, 10)
    R = np.arange(np.prod(shape)).reshape(shape)
    s1, s2, s3 = cd.forward(R, 0)          # slices (u=axis1, v=axis2)
    expect = [R[k, u, v] for k in range(3) for u in range(0, 9, 4) for v in range(0, 10, 4)]
    assert s1.tolist() == expect
    s1b, _, _ = cd.forward(R, 2)           # slices (u=axis0, v=axis1), stacking on the fast axis
    expect_b = [R[u, v, k] for u in range(0, 3, 4) for v in range(0, 9, 4) for k in range(10)]
    assert s1b.tolist() == expect_b


@pytest.mark.parametrize("nu,nv", [(9, 13), (13, 9), (5, 5), (1, 17)])
def test_cd_even_ramp_has_zero_residuals(nu, nv):
    """T = 2*alpha*u + 2*beta*v + gamma is reproduced exactly by floor
    averages, and with axes of 4k+1 points no copy step occurs."""
    u = np.arange(nu)[:, None]
    v = np.arange(nv)[None, :]
    T = (2 * 3 * u - 2 * 5 * v + 11)[None]          # stacked along axis 0
    s1, s2, s3 = cd.forward(T, 0)
    assert np.all(s2 == 0) and np.all(s3 == 0)
    assert s1.size == ((nu + 3) // 4) * ((nv + 3) // 4)


def test_cd_norm_one_exhaustive_line():
    """2D data (slices are lines): any perturbation of the three streams by
    at most 1 moves every recomposed value by at most 1 + 1 + 1, checked
    over every perturbation of a 7-point line."""
    R = np.array([[5, -3, 8, 1, -7, 2, 9]])
    base = cd.forward(R, 0)
    sizes = [s.size for s in base]
    worst = 0
    for pert in itertools.product((-1, 0, 1), repeat=sum(sizes)):
        p = np.array(pert)
        parts = np.split(p, np.cumsum(sizes)[:-1])
        got = cd.inverse([b + q for b, q in zip(base, parts)], R.shape, 0)
        worst = max(worst, int(np.abs(got - R).max()))
    assert worst <= 3


@pytest.mark.parametrize("seed", range(5))
def test_cd_norm_one_random_slices(seed):
    rng = np.random.default_rng(seed)
    shape = (3, 11, 14)
    R = rng.integers(-1000, 1000, size=shape)
    for a in range(3):
        base = cd.forward(R, a)
        E = [int(rng.integers(0, 20)) for _ in range(3)]
        pert = [b + rng.integers(-e, e + 1, size=b.size) for b, e in zip(base, E)]
        got = cd.inverse(pert, shape, a)
        assert np.abs(got - R).max() <= sum(E)


# ------------------------------------------------------------------ codec

def _scalar_encode(q):
    """Pure-Python re-implementation of the written layout."""
    q = [int(v) for v in q]
    n = len(q)
    mags = [abs(v) for v in q]
    B = max(mags).bit_length() if n else 0
    M = (n + 63) // 64
    C = (n + 4095) // 4096
    index, magw, signw = [], [], []
    for j in range(B):
        b = B - 1 - j
        words = [0] * M
        for i, m in enumerate(mags):
            if (m >> b) & 1:
                words[i // 64] |= 1 << (i % 64)
        magw.extend(words)
        sig = [i for i, m in enumerate(mags) if m.bit_length() == b + 1]
        for c in range(C):
            index.append(sum(1 for i in sig if i < 4096 * c))
        sw = [0] * ((len(sig) + 63) // 64)
        for r, i in enumerate(sig):
            if q[i] < 0:
                sw[r // 64] |= 1 << (r % 64)
        signw.extend(sw)
    out = b"".join(v.to_bytes(4, "little") for v in index)
    out += b"\0" * ((-len(out)) % 8)
    out += b"".join(w.to_bytes(8, "little") for w in magw)
    out += b"".join(w.to_bytes(8, "little") for w in signw)
    return out


@pytest.mark.parametrize("n,span", [(0, 1), (1, 5), (63, 100), (64, 2**20), (65, 3), (200, 2**29), (512, 7), (4097, 50)])
def test_codec_bytes_match_scalar_layout(n, span):
    rng = np.random.default_rng(n)
    q = rng.integers(-span, span + 1, size=n)
    q[::7] = 0
    blob, meta = bitplane.encode(q)
    assert blob == _scalar_encode(q)
    assert meta.B == (int(np.abs(q).max()).bit_length() if n else 0)


@pytest.mark.parametrize("n", [1, 70, 512, 5000])
def test_codec_decode_every_k_is_truncation(n):
    rng = np.random.default_rng(7 + n)
    q = (rng.standard_normal(n) * 1000).astype(np.int64) * rng.integers(1, 50, size=n)
    blob, meta = bitplane.encode(q)
    for k in range(meta.B + 1):
        got = bitplane.decode(blob, meta, k)
        np.testing.assert_array_equal(got, bitplane.truncate(q, meta.B, k))
        err = np.abs(got - q).max()
        assert err <= meta.delta(k)
        if k == 0:
            assert err == meta.delta(0)
    np.testing.assert_array_equal(bitplane.decode(blob, meta, meta.B), q)


def test_codec_plane_bytes_and_index():
    rng = np.random.default_rng(3)
    q = rng.integers(-1000, 1000, size=9000)
    blob, meta = bitplane.encode(q)
    _, moff, soff = bitplane.section_offsets(meta)
    assert len(blob) == soff + 8 * sum((s + 63) // 64 for s in meta.nsig)
    idx = bitplane.read_index(blob, meta)
    blen = bitplane.bitlength(np.abs(q))
    for j in range(meta.B):
        b = meta.B - 1 - j
        for c in range(meta.chunks):
            assert idx[j, c] == int((blen[: 4096 * c] == b + 1).sum())
        assert meta.plane_bytes(j) == 4 * 3 + 8 * ((9000 + 63) // 64) + 8 * ((meta.nsig[j] + 63) // 64)


def test_delta_is_strictly_decreasing():
    m = bitplane.StreamMeta(n=10, B=6, maxabs=37, nsig=[1] * 6)
    d = [m.delta(k) for k in range(7)]
    assert d == [37, 31, 15, 7, 3, 1, 0]
