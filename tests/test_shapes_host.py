"""Host logic of the covariance products' launch shapes, through the C ABI without a device
(gp_shape_query): which shape a product takes by default, its padded column count and the
size of its partial sums, against the rules the library states for them, restated here."""
import pytest

from paper_1501_05427_amd import binding as pb

SYM = pb.SHAPE_SYM
TILE = 256      # rows of a row tile; n is padded to a multiple of it
CHUNK = 64      # columns of K per stage; split-K chunks are multiples of it


def n_pad(n):
    return -(-n // TILE) * TILE


def mp_of(m, prec, sym):
    """Padded column count: 4-column groups below 16 (16 for the padded symmetric block),
    16-column MFMA blocks above, in FP32 with up to three (four below 32) columns past a
    block taken on the VALU (mp = 16 floor(m / 16) + 4)."""
    if m < 16:
        return 16 if sym else -(-m // 4) * 4
    t = m % 16
    if prec == pb.GP_FP32 and m < 64 and t and (t <= 3 or (t == 4 and m < 32)):
        return m // 16 * 16 + 4
    return -(-m // 16) * 16


def sym_items(nt, nch, cs):
    return sum(min(nt, (k + 1) * (cs // TILE)) for k in range(nch))


def sym_partial_floats(n, m, prec):
    """(1 + nch + nt) planes of mp x n_pad: the result, the forward partials of the column
    chunks and the transposed partials of the row tiles; the column chunk is the widest of
    512, 1024, 2048 that still gives 2048 work items (else 256)."""
    npd = n_pad(n)
    nt = npd // TILE
    cs = TILE
    c = 2 * TILE
    while c <= 8 * TILE and c <= npd:
        if sym_items(nt, -(-npd // c), c) >= 2048:
            cs = c
        c *= 2
    nch = -(-npd // cs)
    return (1 + nch + nt) * mp_of(m, prec, True) * npd


def split_k(n, m, d, prec, target):
    """Split-K factor for about `target` workgroups: row tiles of 256 rows (VALU, or MFMA at
    d <= 8) or 128 rows (MFMA at d > 8); a factor of 8 or more rounded down to a multiple of 8;
    chunks a multiple of 64 columns."""
    npd = n_pad(n)
    rows = TILE if (m < 16 or d <= 8) else 128
    tiles = npd // rows
    split = min(max(1, target // tiles), npd // CHUNK)
    if split >= 8:
        split = split // 8 * 8
    chunk = -(-(-(-npd // split)) // CHUNK) * CHUNK
    return -(-npd // chunk)


@pytest.mark.parametrize("n,d,m,prec,sym", [
    (65536, 8, 32, pb.GP_FP32, True),          # the benchmark product
    (16384, 8, 17, pb.GP_FP32, True),          # one MFMA block + a VALU column
    (16384, 8, 32, pb.GP_FP32, False),         # two blocks below n = 32768: split-K
    (32768, 8, 32, pb.GP_FP32, True),
    (16384, 16, 32, pb.GP_FP32, True),         # d >= 12: wherever it applies
    (65536, 8, 32, pb.GP_BF16_SPLIT_V, True),  # BF16: two blocks from n = 32768
    (16384, 8, 32, pb.GP_BF16_SPLIT_KV, False),
    (65536, 8, 48, pb.GP_FP32, False),         # three blocks: never symmetric
    (16384, 8, 5, pb.GP_FP32, True),           # under 16 columns: m + d >= 12, n >= 16129
    (16384, 8, 3, pb.GP_FP32, False),
    (16384, 2, 5, pb.GP_FP32, False),
    (16384, 2, 10, pb.GP_FP32, True),
    (16128, 8, 5, pb.GP_FP32, False),
    (65536, 8, 1, pb.GP_FP32, False),
    (131072, 16, 1, pb.GP_FP32, True),
    (65536, 8, 5, pb.GP_BF16_SPLIT_KV, False),  # BF16 under 16 columns: the FP32 VALU product
    (1700, 8, 17, pb.GP_FP32, False),           # fewer than 8 row tiles
    (212000, 8, 32, pb.GP_FP32, True),          # partials just under 24 GiB
    (215000, 8, 32, pb.GP_FP32, False),         # and just over
])
def test_default_shape_and_partials(n, d, m, prec, sym):
    code, split, mp, floats = pb.gp_shape_query(n, d, m, prec)
    assert (code == SYM) == sym, (code, split)
    assert mp == mp_of(m, prec, sym)
    if sym:
        assert split == 1
        assert floats == sym_partial_floats(n, m, prec)
        assert floats * 4 <= 24 << 30
    else:
        target = code
        assert target > 0
        assert split == split_k(n, m, d, prec, target)
        assert floats == split * mp * n_pad(n)


def test_partials_cap_sits_where_stated():
    # the symmetric shape stops where its partials pass 24 GiB (about n = 213000 at m = 32)
    assert sym_partial_floats(212000, 32, pb.GP_FP32) * 4 <= 24 << 30 < sym_partial_floats(215000, 32, pb.GP_FP32) * 4
    with pytest.raises(RuntimeError, match="symmetric"):
        pb.gp_shape_query(215000, 8, 32, code=SYM)


def test_pinned_codes_and_refusals():
    # a split-K code gives that split whatever the default; the symmetric code where it applies
    code, split, mp, floats = pb.gp_shape_query(65536, 8, 32, code=2048)
    assert code == 2048 and split == split_k(65536, 32, 8, pb.GP_FP32, 2048) and floats == split * 32 * 65536
    assert pb.gp_shape_query(16384, 2, 5, code=SYM)[:3] == (SYM, 1, 16)
    for n, d, m, prec in [(1000, 4, 16, pb.GP_FP32), (4000, 4, 18, pb.GP_FP32), (4000, 4, 48, pb.GP_FP32),
                          (4000, 4, 16, pb.GP_BF16_SPLIT_KV), (4000, 4, 5, pb.GP_BF16_SPLIT_V)]:
        with pytest.raises(RuntimeError, match="symmetric"):
            pb.gp_shape_query(n, d, m, prec, code=SYM)
    for args in [(0, 4, 16), (4000, 0, 16), (4000, 17, 16), (4000, 4, 0), (4000, 4, 65)]:
        with pytest.raises(RuntimeError):
            pb.gp_shape_query(*args)
    with pytest.raises(RuntimeError):
        pb.gp_shape_query(4000, 4, 16, code=2 ** 21)
