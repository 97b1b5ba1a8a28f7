"""CPU check of the FP8 tile kernel's direct global->LDS load addresses.

k_tile_fp8 (paper_1603_09596_amd/csrc/tile8.hip) stages 128-byte k slices of
the query rows (Q8, 256 per block) and point rows (X8, 128 per tile) into
three LDS stage buffers with direct loads: instruction j of wave w has lane l
read 16 bytes of row 8 (w + 8 j) + l / 8, k unit (l % 8) ^ (l / 8), at byte
offset row * ld8 + 128 kc + 16 unit from the block's or tile's first row
(rows past the queries or points clamped to that first row, units past the
row to unit 0), and write them at LDS byte buffer + (w + 8 j) * 1 KiB + 16 l.
This test recomputes every offset for ragged sizes and asserts that each read
lies inside Q8 or X8 and each write inside its stage buffer, that each
stage's writes cover the buffer exactly once, and that the MFMA operand reads
find unit u of row r at position u ^ (r & 7).  No GPU."""
import numpy as np
import pytest

KW, KQB, KTP8, KKS8, NWAVES, NBUF = 64, 256, 128, 128, 8, 3
KDMA_A = KQB * KKS8 // 1024 // NWAVES      # 4
KDMA_B = KTP8 * KKS8 // 1024 // NWAVES     # 2
LDS_BYTES = NBUF * (KQB + KTP8) * KKS8 + KQB * 16 + KQB * 4 + KQB * 4 + 2 * KTP8 * 4


def dma_rows_units(j):
    lane = np.arange(KW)
    drow = lane >> 3
    du = (lane & 7) ^ drow
    return drow, du, lane


@pytest.mark.parametrize("ld8", [16, 112, 128, 144, 1008, 10000])
@pytest.mark.parametrize("nq,n", [(1, 1), (255, 127), (256, 128), (257, 129), (2000, 200_000)])
def test_loads_stay_inside_rows_and_stage_buffers(ld8, nq, n):
    nk = (ld8 + KKS8 - 1) // KKS8
    nqb = (nq + KQB - 1) // KQB
    ntiles = (n + KTP8 - 1) // KTP8
    for qblk in sorted({0, nqb - 1}):
        q0 = qblk * KQB
        for it in sorted({0, ntiles - 1}):
            x0 = it * KTP8
            for kc in sorted({0, nk - 1}):
                seenA = np.zeros(KQB * KKS8 // 16, int)
                seenB = np.zeros(KTP8 * KKS8 // 16, int)
                for w in range(NWAVES):
                    drow, du, lane = dma_rows_units(0)
                    k = KKS8 * kc + 16 * du
                    koff = np.where(k < ld8, k, 0)
                    for j in range(KDMA_A):
                        r = 8 * (w + 8 * j) + drow
                        rr = np.where(q0 + r < nq, r, 0)
                        g = (q0 + rr) * ld8 + koff
                        assert g.min() >= 0 and (g + 16).max() <= nq * ld8
                        lds = (w + 8 * j) * 1024 + 16 * lane
                        assert (lds + 16).max() <= KQB * KKS8
                        seenA[lds // 16] += 1
                        # the unit written at LDS row r, position p is unit p ^ (r & 7)
                        p = (lds % KKS8) // 16
                        assert ((lds // KKS8) == r).all() and (du == (p ^ (r & 7))).all()
                    for j in range(KDMA_B):
                        r = 8 * (w + 8 * j) + drow
                        rr = np.where(x0 + r < n, r, 0)
                        g = (x0 + rr) * ld8 + koff
                        assert g.min() >= 0 and (g + 16).max() <= n * ld8
                        lds = (w + 8 * j) * 1024 + 16 * lane
                        assert (lds + 16).max() <= KTP8 * KKS8
                        seenB[lds // 16] += 1
                assert (seenA == 1).all() and (seenB == 1).all()


def test_operand_reads_find_their_units():
    """Lane (fg, fr) of fragment i reads units 2 fg and 2 fg + 1 of row
    16 i + fr (+ 64 per wave block) at positions u ^ (r & 7)."""
    for r in range(KQB):
        for fg in range(4):
            for u in (2 * fg, 2 * fg + 1):
                pos = u ^ (r & 7)
                assert 0 <= pos < 8
                assert (pos ^ (r & 7)) == u


def test_static_lds_allocation_fits():
    assert LDS_BYTES == 154_624
    assert LDS_BYTES <= 160 * 1024
