"""ORACLE — test infrastructure only: the BLCO encoding written out step by step.

Follows Section 4 of the paper: ALTO linearization of the coordinates
(Section 4.1, Figure 6a), ordering of the non-zeros along the encoding line,
re-encoding of the linear index into contiguous per-mode bit fields decoded by
shift and mask (Section 4.1, Figure 6b), and adaptive blocking on the
uppermost bits when the encoding line needs more than the target integer width,
followed by splitting blocks to a maximum non-zero count (Section 4.2).

Readings taken where the paper leaves a convention open (each is also listed
with the design notes):
  * bits of mode n: b_n = ceil(log2 I_n), 0 when I_n = 1;
  * ALTO bit order for irregular shapes: round robin over the modes from the
    least significant bit, mode 1 first at each level, a mode dropping out once
    its bits are used up (for equal widths this is Morton order);
  * the block key is the top T - K bits of the ALTO index, K = min(T, key_bits);
  * re-encoded key: mode 1's kept bits in the least significant field, fields
    ascending by mode;
  * order inside a block: ALTO order (not key order);
  * a block larger than max_block_nnz is split front to back into chunks.

Linear indices may need up to 128 bits; they are held as two uint64 arrays
(lo = bits 0..63, hi = bits 64..127).  Nothing here is shared with the library.
"""
from __future__ import annotations

import numpy as np


def bit_widths(dims):
    """b_n = number of bits needed for indices 0..I_n-1."""
    out = []
    for I in dims:
        I = int(I)
        b = 0
        while (1 << b) < I:
            b += 1
        out.append(b)
    return out


def alto_positions(b):
    """pos[n][j] = position on the encoding line of bit j of mode n.

    Levels j = 0, 1, ... from the least significant bit; inside a level the
    modes take the next free position in order 1..N, skipping modes whose
    bits are exhausted (recursive halving of the longest modes).
    """
    pos = [[0] * bn for bn in b]
    p = 0
    for j in range(max(b) if b else 0):
        for n, bn in enumerate(b):
            if j < bn:
                pos[n][j] = p
                p += 1
    return pos


def linearize(coords, pos):
    """ALTO linear index of every non-zero as (lo, hi) uint64 arrays."""
    nnz = len(coords[0]) if coords else 0
    lo = np.zeros(nnz, dtype=np.uint64)
    hi = np.zeros(nnz, dtype=np.uint64)
    for n, pn in enumerate(pos):
        c = coords[n].astype(np.uint64)
        for j, p in enumerate(pn):
            bit = (c >> np.uint64(j)) & np.uint64(1)
            if p < 64:
                lo |= bit << np.uint64(p)
            else:
                hi |= bit << np.uint64(p - 64)
    return lo, hi


def _shift_right(lo, hi, K):
    """(hi:lo) >> K as uint64 (the caller guarantees the result fits)."""
    if K == 0:
        assert not np.any(hi)
        return lo.copy()
    if K < 64:
        return (lo >> np.uint64(K)) | (hi << np.uint64(64 - K))
    return hi >> np.uint64(K - 64)


def layout(dims, key_bits=64):
    """The bit map: widths, positions, kept/stripped split, field shifts."""
    b = bit_widths(dims)
    T = sum(b)
    K = min(T, key_bits)
    pos = alto_positions(b)
    h = [sum(1 for p in pn if p >= K) for pn in pos]   # bits of mode n moved to the block key
    w = [bn - hn for bn, hn in zip(b, h)]              # bits of mode n kept in the key
    s = []
    acc = 0
    for wn in w:
        s.append(acc)
        acc += wn
    return dict(b=b, T=T, K=K, pos=pos, h=h, w=w, s=s, S=T - K)


def encode(coords, vals, dims, key_bits=64, max_block_nnz=1 << 27):
    """BLCO tensor of a COO tensor.

    Returns keys (uint64), values (float32, permuted), block_ids (uint64),
    block_starts (int64, nblocks + 1), the layout and the permutation applied.
    """
    lay = layout(dims, key_bits)
    if lay["S"] > 64:
        raise ValueError("block key wider than 64 bits")
    nnz = len(vals)
    lo, hi = linearize(coords, lay["pos"])
    order = np.lexsort((lo, hi))            # stable; hi is the major key
    lo, hi = lo[order], hi[order]
    blk = _shift_right(lo, hi, lay["K"])    # uppermost T - K bits
    del lo, hi
    keys = np.zeros(nnz, dtype=np.uint64)
    for n, c in enumerate(coords):
        field = c[order].astype(np.uint64) & np.uint64((1 << lay["w"][n]) - 1)
        keys |= field << np.uint64(lay["s"][n])
    # blocks: maximal runs of equal block key, each split front to back
    if nnz:
        run_start = np.flatnonzero(np.concatenate([[True], blk[1:] != blk[:-1]]))
    else:
        run_start = np.zeros(0, dtype=np.int64)
    run_end = np.concatenate([run_start[1:], [nnz]]).astype(np.int64)
    ids, starts = [], []
    for a, e in zip(run_start.tolist(), run_end.tolist()):
        for c0 in range(a, e, max_block_nnz):
            ids.append(int(blk[a]))
            starts.append(c0)
    starts.append(nnz)
    return dict(keys=keys, values=np.asarray(vals, dtype=np.float32)[order],
                block_ids=np.asarray(ids, dtype=np.uint64),
                block_starts=np.asarray(starts, dtype=np.int64), layout=lay, order=order)


def block_high_bits(block_id, lay, n):
    """hi_n(B): the bits of block key B that belong to mode n, in mode n's bit order."""
    out = 0
    K = lay["K"]
    for t in range(lay["h"][n]):
        p = lay["pos"][n][lay["w"][n] + t]
        out |= ((int(block_id) >> (p - K)) & 1) << t
    return out


def decode(keys, block_ids, block_starts, lay):
    """Coordinates back from (key, block): field by shift and mask, top bits from the block."""
    N = len(lay["b"])
    nnz = len(keys)
    coords = [np.zeros(nnz, dtype=np.uint64) for _ in range(N)]
    for bi in range(len(block_ids)):
        a, e = int(block_starts[bi]), int(block_starts[bi + 1])
        kk = keys[a:e]
        for n in range(N):
            field = (kk >> np.uint64(lay["s"][n])) & np.uint64((1 << lay["w"][n]) - 1)
            top = np.uint64(block_high_bits(block_ids[bi], lay, n) << lay["w"][n])
            coords[n][a:e] = field | top
    return [c.astype(np.uint32) for c in coords]
