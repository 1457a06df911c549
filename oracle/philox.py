"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written from the published definition.

TEST INFRASTRUCTURE ONLY (see the package header).

One Philox round maps the counter (c0, c1, c2, c3) with key (k0, k1) to
(hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); the key is
bumped by the Weyl constants (W0, W1) between rounds; ten rounds.

Stream layout used by the sweep (shared convention with the HIP library; each
side implements it independently):

* key = (lo32(seed), hi32(seed) XOR tag), tag INIT = 0 (initial field),
  ACCEPT = 1 (Metropolis draws);
* counter = (chain, sweep, slice, site);
* uniform u = ((w0 >> 5) * 2**26 + (w1 >> 6)) * 2**-53, in [0, 1) with 53 bits.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF

TAG_INIT = 0
TAG_ACCEPT = 1


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ``ctr``: integer array of shape (..., 4) (uint32 values); ``key``: 2 ints.
    Returns a uint64 array of shape (..., 4) holding the four 32-bit words.
    """
    c = np.asarray(ctr, dtype=np.uint64) & np.uint64(MASK)
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0 = np.uint64(int(key[0]) & MASK)
    k1 = np.uint64(int(key[1]) & MASK)
    m = np.uint64(MASK)
    s32 = np.uint64(32)
    for _ in range(10):
        p0 = np.uint64(M0) * c0          # < 2**64: exact in uint64
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> s32, p0 & m
        hi1, lo1 = p1 >> s32, p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & m
        k1 = (k1 + np.uint64(W1)) & m
    return np.stack([c0, c1, c2, c3], axis=-1)


def stream_key(seed: int, tag: int):
    seed = int(seed)
    return (seed & MASK, ((seed >> 32) & MASK) ^ int(tag))


def uniform53(words):
    """Map the first two words to a 53-bit uniform double in [0, 1)."""
    w0 = np.asarray(words[..., 0], dtype=np.uint64)
    w1 = np.asarray(words[..., 1], dtype=np.uint64)
    a = (w0 >> np.uint64(5)).astype(np.float64)
    b = (w1 >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0)


def accept_uniforms(seed: int, chain: int, sweep: int, slice_: int, n_sites: int):
    """Metropolis uniforms for every site of one slice of one sweep."""
    i = np.arange(n_sites, dtype=np.uint64)
    ctr = np.stack([np.full_like(i, chain), np.full_like(i, sweep),
                    np.full_like(i, slice_), i], axis=-1)
    return uniform53(philox4x32_10(ctr, stream_key(seed, TAG_ACCEPT)))


def initial_field(seed: int, chain: int, n_slices: int, n_sites: int):
    """Initial Ising field: s = +1 where bit 0 of word 0 is set, else -1."""
    l, i = np.meshgrid(np.arange(n_slices, dtype=np.uint64),
                       np.arange(n_sites, dtype=np.uint64), indexing="ij")
    ctr = np.stack([np.full_like(l, chain), np.zeros_like(l), l, i], axis=-1)
    w = philox4x32_10(ctr, stream_key(seed, TAG_INIT))
    return np.where((w[..., 0] & np.uint64(1)) == 1, 1, -1).astype(np.int8)
