"""The window argument of the gradient's LDS-tiled adjoint, on the CPU.

Each 16 x 16 block stages psi on rows y0 - 2r .. y0 + 16 + 3r - 1 (and the
same columns), in rows of 48 floats.  A pixel y of the block sums over its
mirrored extended rows s (y itself, -1-y for y < r, 2H-1-y for y >= H-r) and
reads q = s - a + r for a = 0 .. 2r.  Checked exhaustively here: every such q
falls inside the staged window, so the tile index is in bounds and the
padded row stride never wraps into the next row."""
import pytest

KB = 16


def tile_shape(r):
    th = tw = KB + 5 * r
    ts = (tw + 16 + 31) // 32 * 32 - 16
    return th, tw, ts


@pytest.mark.parametrize("r", [1, 2, 3])
def test_every_tap_read_stays_in_the_staged_window(r):
    th, tw, ts = tile_shape(r)
    assert ts >= tw and ts % 32 == 16
    for n in range(r, 200):                       # image height (or width)
        for b0 in range(0, n, KB):                # block origin
            for y in range(b0, min(b0 + KB, n)):
                rows = [y] + ([-1 - y] if y < r else []) + ([2 * n - 1 - y] if y >= n - r else [])
                for s in rows:
                    assert b0 - r <= s < b0 + KB + 2 * r
                    for a in range(2 * r + 1):
                        t = s - b0 + 3 * r - a    # tile row (or column) of q
                        assert 0 <= t < th
                        assert b0 - 2 * r + t == s - a + r


@pytest.mark.parametrize("r", [1, 2, 3])
def test_padded_rows_spread_a_wave_over_the_banks(r):
    """The four 16-lane rows of a wave read 64 distinct banks (and, on 32
    banks, each bank exactly twice, the minimum for 64 lanes)."""
    _, _, ts = tile_shape(r)
    for base in range(0, 64):
        banks64 = {(base + row * ts + lane) % 64 for row in range(4) for lane in range(16)}
        assert len(banks64) == 64
        counts32 = [0] * 32
        for row in range(4):
            for lane in range(16):
                counts32[(base + row * ts + lane) % 32] += 1
        assert max(counts32) == 2
