"""Index maps of the pre-pass images (layout only, no arithmetic of the method): turn the panel
images a variant writes back into plain row-major arrays, following the layout that
include/compar.h documents for cmp_prepass_images."""
import numpy as np


def panel_gather_index(rows: int, kbytes: int) -> np.ndarray:
    """Byte offset of (row, kbyte) in a panel image of `rows` rows (a multiple of 256) and
    `kbytes` bytes of K per row (a multiple of 64): 256-row x 64-byte blocks of 16 KiB, the
    K extent of a panel contiguous, 16-byte chunk c of row r stored at c ^ ((r / 4) % 4)."""
    r = np.arange(rows, dtype=np.int64)[:, None]
    kb = np.arange(kbytes, dtype=np.int64)[None, :]
    nkb = kbytes // 64
    rr = r % 256
    chunk = ((kb // 16) % 4) ^ ((rr // 4) % 4)
    return ((r // 256) * nkb + kb // 64) * 16384 + rr * 64 + chunk * 16 + kb % 16


def unpack_panel_bytes(img: np.ndarray, rows: int, kbytes: int) -> np.ndarray:
    """rows x kbytes uint8 array of a panel image."""
    return np.asarray(img, np.uint8)[panel_gather_index(rows, kbytes)]


def unpack_panel_bf16(img: np.ndarray, rows: int, kp: int) -> np.ndarray:
    """rows x kp uint16 bit patterns of a bf16 panel image (2 bytes per value, little endian)."""
    b = unpack_panel_bytes(img, rows, 2 * kp).astype(np.uint16)
    return b[:, 0::2] | (b[:, 1::2] << 8)


def unpack_mx6_codes(img: np.ndarray, rows: int, kp: int) -> np.ndarray:
    """rows x kp E2M3 codes (uint8, 6 bits) of an MX FP6 code image: per 256-row x 64-value
    block, 48 bytes per row [half 0 bytes 0-15 | half 1 bytes 0-15 | half 0 bytes 16-23 |
    half 1 bytes 16-23]; the 32 codes of a half packed 6 bits each, code j at bit 6 j."""
    img = np.asarray(img, np.uint8)
    nkb = kp // 64
    r = np.arange(rows, dtype=np.int64)[:, None, None, None]
    kb = np.arange(nkb, dtype=np.int64)[None, :, None, None]
    h = np.arange(2, dtype=np.int64)[None, None, :, None]
    byte = np.arange(24, dtype=np.int64)[None, None, None, :]
    pos = np.where(byte < 16, 16 * h + byte, 32 + 8 * h + (byte - 16))
    off = ((r // 256) * nkb + kb) * (256 * 48) + (r % 256) * 48 + pos
    raw = img[off]                                    # rows x nkb x 2 x 24 bytes
    bits = np.unpackbits(raw, axis=-1, bitorder="little")     # rows x nkb x 2 x 192 bits
    bits = bits.reshape(rows, nkb, 2, 32, 6)
    weights = (1 << np.arange(6)).astype(np.uint8)
    codes = (bits * weights).sum(axis=-1).astype(np.uint8)    # code j from bits 6j .. 6j+5
    return codes.reshape(rows, kp)


def unpack_mx6_scales(img: np.ndarray, rows: int, kp: int):
    """(hi, lo) E8M0 scale bytes, rows x (kp / 32) each, of an MX FP6 scale image: per 256-row
    x 64-value block a 1 KiB block, 4 bytes per row (half 0 hi, half 0 lo, half 1 hi,
    half 1 lo)."""
    img = np.asarray(img, np.uint8)
    nkb = kp // 64
    r = np.arange(rows, dtype=np.int64)[:, None, None]
    kb = np.arange(nkb, dtype=np.int64)[None, :, None]
    h = np.arange(2, dtype=np.int64)[None, None, :]
    base = ((r // 256) * nkb + kb) * 1024 + (r % 256) * 4 + 2 * h
    return img[base].reshape(rows, 2 * nkb), img[base + 1].reshape(rows, 2 * nkb)
