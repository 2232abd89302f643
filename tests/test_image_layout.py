"""CPU checks of the test-side index maps of the pre-pass images (tests/image_layout.py): each
is a bijection onto the image bytes, hand-computed offsets, and the MX FP6 unpacking inverts a
packing written bit by bit from the documented layout."""
import numpy as np

from image_layout import (panel_gather_index, unpack_mx6_codes, unpack_mx6_scales,
                          unpack_panel_bf16, unpack_panel_bytes)


def test_panel_index_is_a_bijection():
    for rows, kbytes in [(256, 64), (512, 192), (256, 1024)]:
        idx = panel_gather_index(rows, kbytes)
        assert np.array_equal(np.sort(idx.ravel()), np.arange(rows * kbytes))


def test_panel_index_hand_values():
    idx = panel_gather_index(512, 128)
    assert idx[0, 0] == 0 and idx[0, 17] == 17
    assert idx[4, 0] == 4 * 64 + 16           # row 4: chunk 0 stored at position 1
    assert idx[4, 16] == 4 * 64 + 0           # chunk 1 at position 0
    assert idx[13, 40] == 13 * 64 + (2 ^ 3) * 16 + 8
    assert idx[0, 64] == 16384                # second K block of panel 0
    assert idx[256, 0] == 2 * 16384           # panel 1 follows both K blocks of panel 0


def test_panel_bf16_little_endian():
    img = np.zeros(256 * 128, np.uint8)
    img[0], img[1] = 0x80, 0x3F               # value (0, 0) = 0x3f80 (1.0)
    v = unpack_panel_bf16(img, 256, 64)
    assert v[0, 0] == 0x3F80 and v.shape == (256, 64) and np.count_nonzero(v) == 1
    assert unpack_panel_bytes(img, 256, 128)[0, 1] == 0x3F


def test_mx6_unpack_inverts_a_bit_by_bit_packing():
    rows, kp = 512, 128
    g = np.random.default_rng(0)
    codes = g.integers(0, 64, size=(rows, kp)).astype(np.uint8)
    sh = g.integers(0, 256, size=(rows, kp // 32)).astype(np.uint8)
    sl = g.integers(0, 256, size=(rows, kp // 32)).astype(np.uint8)
    nkb = kp // 64
    code_img = np.zeros(rows // 256 * nkb * 256 * 48, np.uint8)
    scale_img = np.zeros(rows // 256 * nkb * 1024, np.uint8)
    for r in range(rows):
        for kb in range(nkb):
            for h in range(2):
                word = 0
                for j in range(32):
                    word |= int(codes[r, 64 * kb + 32 * h + j]) << (6 * j)
                half = word.to_bytes(24, "little")
                blk = ((r // 256) * nkb + kb) * 256 * 48 + (r % 256) * 48
                code_img[blk + 16 * h: blk + 16 * h + 16] = list(half[:16])
                code_img[blk + 32 + 8 * h: blk + 40 + 8 * h] = list(half[16:])
                s = ((r // 256) * nkb + kb) * 1024 + (r % 256) * 4 + 2 * h
                scale_img[s] = sh[r, 2 * kb + h]
                scale_img[s + 1] = sl[r, 2 * kb + h]
    assert np.array_equal(unpack_mx6_codes(code_img, rows, kp), codes)
    gh, gl = unpack_mx6_scales(scale_img, rows, kp)
    assert np.array_equal(gh, sh) and np.array_equal(gl, sl)
