"""CPU check of the FP8 tile kernel's direct global->LDS load addresses.

k_tile_fp8 (paper_1603_09596_amd/csrc/tile8.hip) stages 64-byte k slices of
the query rows (Q8, 256 per block) and point rows (X8, 256 per pair of
128-point tiles) into four LDS stage buffers with direct loads.  Rows are
paired into 128-byte lines: row r lives in line r >> 1, its 16-byte unit u at
position (u + 4 (r & 1)) ^ ((r >> 1) & 7).  Instruction j of wave w writes
lines 8 (w + 8 j) .. + 8; lane l writes position l % 8 of line
8 (w + 8 j) + l / 8 and so reads row 2 line + s / 4, unit s % 4, with
s = (l % 8) ^ (l / 8), at byte offset row * ld8 + 64 kc + 16 unit from the
block's or pair's first row (rows past the queries or points clamped to that
first row, units past the row to unit 0).  This test recomputes every offset
for ragged sizes and asserts that each read lies inside Q8 or X8, each write
inside its stage buffer, that each stage's writes cover the buffer exactly
once with the layout the operand reads assume, and that the operand reads of
8 consecutive rows fall on 8 different 16-byte bank groups.  No GPU."""
import numpy as np
import pytest

KW, KQB, KTW, KKS, NWAVES, NBUF = 64, 256, 256, 64, 8, 4
KDMA_A = KQB * KKS // 1024 // NWAVES      # 2
KDMA_B = KTW * KKS // 1024 // NWAVES      # 2
LDS_BYTES = NBUF * (KQB + KTW) * KKS + KQB * 2 * 2 * 8 + KQB * 2 * 4 + KQB * 4 + 2 * KTW * 4


def unit_off(r, u):
    return (r >> 1) * 128 + (((u + 4 * (r & 1)) ^ ((r >> 1) & 7)) << 4)


def dma_lane():
    lane = np.arange(KW)
    dline = lane >> 3
    ds = (lane & 7) ^ dline
    return lane, 2 * dline + (ds >> 2), ds & 3


@pytest.mark.parametrize("ld8", [16, 48, 64, 80, 1008, 10000])
@pytest.mark.parametrize("nq,n", [(1, 1), (255, 127), (256, 256), (257, 300), (2000, 200_000)])
def test_loads_stay_inside_rows_and_stage_buffers(ld8, nq, n):
    nk = (ld8 + KKS - 1) // KKS
    nqb = (nq + KQB - 1) // KQB
    ntiles = (n + 127) // 128
    lane, drow, du = dma_lane()
    for qblk in sorted({0, nqb - 1}):
        q0 = qblk * KQB
        for T in sorted({0, (ntiles - 1) // 2 * 2}):
            x0 = T * 128
            for kc in sorted({0, nk - 1}):
                k = KKS * kc + 16 * du
                koff = np.where(k < ld8, k, 0)
                for rows, base, nrows, cap, ndma in ((KQB, q0, nq, nq, KDMA_A), (KTW, x0, n, n, KDMA_B)):
                    seen = np.zeros(rows * KKS // 16, int)
                    for w in range(NWAVES):
                        for j in range(ndma):
                            r = 16 * (w + 8 * j) + drow
                            rr = np.where(base + r < nrows, r, 0)
                            g = (base + rr) * ld8 + koff
                            assert g.min() >= 0 and (g + 16).max() <= cap * ld8
                            lds = (w + 8 * j) * 1024 + 16 * lane
                            assert (lds + 16).max() <= rows * KKS
                            assert (lds == unit_off(r, du)).all()   # where the operand reads look
                            seen[lds // 16] += 1
                    assert (seen == 1).all()


def test_operand_reads_of_eight_rows_use_eight_bank_groups():
    for r0 in range(0, KQB, 8):
        for u in range(4):
            groups = {(unit_off(r, u) % 128) // 16 for r in range(r0, r0 + 8)}
            assert len(groups) == 8


def test_static_lds_allocation_fits():
    assert LDS_BYTES == 144_384
    assert LDS_BYTES <= 160 * 1024
