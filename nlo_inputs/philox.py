"""Philox4x32-10 counter-based random numbers (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), vectorised in numpy.

A draw is a pure function of (key, counter): event ``e`` of a workload always
receives the same numbers, whatever the batch size, chunking or thread count.
This removes the "shift in random number generation calls" that broke
same-seed agreement between serial and vectorised runs in the paper's
multithreaded prototype (section "Implementation status").
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32(ctr, key, rounds=10):
    """ctr: uint32-valued array [..., 4]; key: uint32-valued [..., 2] (broadcast).

    Returns uint32 array [..., 4].  Each round multiplies words 0 and 2 by the
    two Philox multipliers (full 64-bit product split into hi/lo), swaps and
    xors with the round key; the key is bumped by the Weyl constants between
    rounds.
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(key[..., 0], c0.shape).astype(np.uint64)
    k1 = np.broadcast_to(key[..., 1], c0.shape).astype(np.uint64)
    for r in range(rounds):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def uniforms(seed, stream, event_index, slot):
    """Two independent doubles in (0, 1) per (event, slot).

    key = (seed, stream); counter = (event lo, event hi, slot, 0).  Each double
    takes 53 bits from a pair of 32-bit words and is offset by half an ulp so
    that log(u) is always finite.
    Returns array [len(event_index), 2].
    """
    ev = np.asarray(event_index, dtype=np.uint64)
    ctr = np.zeros(ev.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = ev & _MASK
    ctr[..., 1] = ev >> _S32
    ctr[..., 2] = np.uint64(slot)
    out = philox4x32(ctr, np.array([seed, stream], dtype=np.uint64)).astype(np.uint64)
    a = ((out[..., 0] >> np.uint64(5)) << np.uint64(26)) | (out[..., 1] >> np.uint64(6))
    b = ((out[..., 2] >> np.uint64(5)) << np.uint64(26)) | (out[..., 3] >> np.uint64(6))
    scale = 1.0 / 9007199254740992.0  # 2^-53
    return np.stack([(a.astype(np.float64) + 0.5) * scale,
                     (b.astype(np.float64) + 0.5) * scale], axis=-1)
