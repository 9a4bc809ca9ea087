"""The fused DUGKS step's work split (the z_chunk setting; fused_work_items
and fused_work_item run the library's own item decoder on the host, no GPU
needed).

Every tile-plane of a box must belong to exactly one work item, for plain
z-chunks, for chunks whose last, partly filled round is cut into z-parts laid
out per XCD, and for the automatic choice, over box sizes, tile widths and
device sizes (slots: blocks of the kernel the device holds at once).  The
tiling is re-derived here from its definition (tiles of tile_width - 2 by 6
updated columns, numbered x fastest), not taken from the library.
"""
import math

import pytest

import paper_1601_03815_amd as dhit


def _params(n, precision="fp64", tile=0, chunk=0):
    p = dhit.default_params(n, dhit.DUGKS, dhit.FP64 if precision == "fp64" else dhit.FP32, 0.01)
    p.tile_width = tile
    p.z_chunk = chunk
    return p


def _cover(p, slots):
    """Checks the partition; returns (items, z_chunk in effect, [(tile, z0, planes)])."""
    n = p.n
    w = p.tile_width or 32
    tiles = math.ceil(n / (w - 2)) * math.ceil(n / 6)
    items, zc = dhit.fused_work_items(p, slots)
    seen = set()
    split = []
    for it in range(items):
        t, z0, k = dhit.fused_work_item(p, slots, it)
        split.append((t, z0, k))
        if k == 0:
            continue
        assert 0 <= t < tiles and 0 <= z0 and z0 + k <= n, (n, w, p.z_chunk, slots, it, t, z0, k)
        for z in range(z0, z0 + k):
            assert (t, z) not in seen, (n, w, p.z_chunk, slots, it, t, z)
            seen.add((t, z))
    assert len(seen) == tiles * n, (n, w, p.z_chunk, slots)
    return items, zc, split


@pytest.mark.parametrize("n", [4, 5, 17, 40, 64, 97])
@pytest.mark.parametrize("tile", [16, 32])
def test_every_tile_plane_once(n, tile):
    for chunk in sorted({0, 1, 2, 5, 7, n, -1, -2, -3, -5, -7, -n}):
        if abs(chunk) > n:
            continue
        for slots in (64, 256, 512, 1024):
            _cover(_params(n, tile=tile, chunk=chunk), slots)


def test_plain_chunks_are_tiles_by_chunks():
    """z_chunk = c > 0: one item per tile and chunk, tile fastest."""
    p = _params(256, chunk=37)
    items, zc, split = _cover(p, 256)
    assert (items, zc) == (387 * 7, 37)
    assert split[0] == (0, 0, 37) and split[386] == (386, 0, 37) and split[387] == (0, 37, 37)
    assert split[-1] == (386, 222, 34)


def test_automatic_choice_at_256():
    """At 256^3 on a 256-unit device: FP64 (one block per unit) takes
    128-plane chunks with the last round cut (3 full rounds of 256 chunks,
    6 chunks left, each cut into 32 parts of 4 planes: up to 42 parts would
    fit the round, and 4 planes is the length that needs), FP32 (two blocks
    per unit) 64-plane chunks cut (3 full rounds of 512, 12 chunks left in 32
    parts of 2 planes).  Items per XCD: its eighth of the whole chunks, then
    its eighth of the parts."""
    items, zc, split = _cover(_params(256, "fp64"), 256)
    assert zc == -128 and items == 8 * (768 // 8 + math.ceil(6 * 32 / 8))
    parts = [s for s in split if s[2] and s[2] < 128]
    assert len(parts) == 6 * 32 and {s[2] for s in parts} == {4}
    items, zc, split = _cover(_params(256, "fp32"), 512)
    assert zc == -64 and items == 8 * (1536 // 8 + math.ceil(12 * 32 / 8))
    parts = [s for s in split if s[2] and s[2] < 64]
    assert len(parts) == 12 * 32 and {s[2] for s in parts} == {2}


def test_cut_parts_of_neighbouring_tiles_are_consecutive():
    """Within an XCD's eighth, the parts follow its whole chunks and are
    numbered part by part: consecutive items hold neighbouring tiles at the
    same planes."""
    p = _params(256, chunk=-128)
    items, _, split = _cover(p, 256)
    eighth = items // 8
    whole = 768 // 8
    for x in range(8):
        seg = split[x * eighth:(x + 1) * eighth]
        assert all(k == 128 for _, _, k in seg[:whole])
        parts = [s for s in seg[whole:] if s[2]]
        for a, b in zip(parts, parts[1:]):
            assert (b[0] == a[0] + 1 and b[1] == a[1]) or b[1] > a[1] or b[0] < a[0]


def test_no_cut_without_a_full_round():
    """A launch that does not fill one round is left as it is."""
    for chunk in (-5, 5):
        items, zc, _ = _cover(_params(17, chunk=chunk), 256)
        assert items == 3 * 4 and zc == chunk


def test_work_split_errors():
    with pytest.raises(dhit.DhitError):
        dhit.fused_work_items(dhit.default_params(32, dhit.LBE_MRT, dhit.FP64, 0.01), 256)
    with pytest.raises(dhit.DhitError):
        dhit.fused_work_items(_params(32), 0)
    with pytest.raises(dhit.DhitError):
        dhit.fused_work_item(_params(32), 256, 10 ** 6)
    with pytest.raises(dhit.DhitError):
        dhit.fused_work_items(_params(32, chunk=-33), 256)
