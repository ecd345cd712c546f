"""Bit packing of a 0/1 haplotype matrix into variant-major 32-bit words.

Layout (the haplotype cache of section 4.1.1 of the kalis paper, in our own
words): the matrix is stored variant by variant. At each variant the N
alleles are packed 32 haplotypes per unsigned 32-bit word; haplotype j sits
at bit (j mod 32), least significant bit first, of word floor(j/32). Each
variant row is padded to a whole number of 32-byte blocks, so every row starts
on a 32-byte boundary and the tail bits of the last word are unused (zero).

Two consecutive 32-bit words form one little-endian 64-bit word, so bit
(j mod 64) of 64-bit word floor(j/64) is also haplotype j.
"""

from __future__ import annotations

import numpy as np

ROW_ALIGN_WORDS = 8  # 32 bytes


def packed_stride_words(n_haps: int, align_words: int = ROW_ALIGN_WORDS) -> int:
    """Number of 32-bit words per variant row for ``n_haps`` haplotypes."""
    if n_haps < 1:
        raise ValueError("n_haps must be >= 1")
    words = (n_haps + 31) // 32
    return ((words + align_words - 1) // align_words) * align_words


def packed_bytes(n_haps: int, n_variants: int, align_words: int = ROW_ALIGN_WORDS) -> int:
    """Bytes taken by the packed matrix (the cache size)."""
    return 4 * packed_stride_words(n_haps, align_words) * n_variants


def pack_haplotypes(h: np.ndarray, align_words: int = ROW_ALIGN_WORDS,
                    chunk: int = 4096) -> np.ndarray:
    """Pack an L x N 0/1 matrix (variant-major) into an L x stride uint32 array."""
    h = np.asarray(h)
    if h.ndim != 2:
        raise ValueError("h must be 2-D (variants x haplotypes)")
    L, N = h.shape
    stride = packed_stride_words(N, align_words)
    out = np.zeros((L, stride), dtype=np.uint32)
    out_bytes = out.view(np.uint8).reshape(L, stride * 4)
    nbytes = (N + 7) // 8
    for a in range(0, L, chunk):
        b = min(L, a + chunk)
        blk = np.ascontiguousarray(h[a:b] != 0, dtype=np.uint8)
        out_bytes[a:b, :nbytes] = np.packbits(blk, axis=1, bitorder="little")
    return out


def unpack_haplotypes(words: np.ndarray, n_haps: int) -> np.ndarray:
    """Inverse of :func:`pack_haplotypes`: returns an L x N uint8 matrix."""
    words = np.ascontiguousarray(words, dtype=np.uint32)
    L = words.shape[0]
    by = words.view(np.uint8).reshape(L, -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :n_haps].copy()
