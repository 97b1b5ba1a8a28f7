"""CPU check of the BF16 tile kernel's direct global->LDS load addresses.

k_tile_bf16 (paper_1603_09596_amd/csrc/tile.hip) stages rows of X16 and its
epilogue operands into LDS with direct loads whose addresses it computes
itself: per stage, instruction j of wave w has lane l read 16 bytes at byte
offset trow[j] + koff of its split's rows and write them at LDS byte
xs0 + buf * 32 KiB + (w + 8 j) * 1 KiB + 16 l; per tile, waves 0..3 load
the candidate words, the norms and the block's rows of shared bounds (four
words per query: the bound and up to three splits' rank scores) into the
epilogue area, and the two waves of each pair swap partial sums through a
32 KiB exchange area.  This test recomputes those offsets with the kernel's
formulas for every configuration launch_tile_path admits (the row stride,
the template k depth, ragged point counts and splits, query chunkings) and
asserts that every global access lies inside its buffer and every LDS target
inside the kernel's static allocation (3 x 32 KiB stages + two 832-word
epilogue areas, used by alternate tiles, + 32 KiB exchange = 134.5 KiB).
No GPU."""
import numpy as np
import pytest

KTP, KKS, KNBUF, KTWAVES, KWAVE, KTQ = 64, 256, 3, 8, 64, 128
KSTAGE = KTP * KKS * 2                      # bytes per stage
KUNITS = KKS // 8                           # 16-byte units per staged row
KROWS_PER_INST = KWAVE // KUNITS            # rows per 1 KiB wave instruction
KDMA_PER_WAVE = KSTAGE // 1024 // KTWAVES   # 4
KBOUND_WORDS = 4                            # per query: shared bound + 3 rank scores
KEPI_VIS, KEPI_NORM, KEPI_THR = 0, 4 * KTP, 5 * KTP
KEPI_WORDS = 5 * KTP + KBOUND_WORDS * KTQ
KXCH_BYTES = KTWAVES * 4 * KWAVE * 16      # f4 partial sums [wave][block][lane]
KEPI_BUFS = 2                               # tile t's operands go to area t & 1
LDS_BYTES = KNBUF * KSTAGE + KEPI_BUFS * 4 * KEPI_WORDS + KXCH_BYTES
KSTEPS_TEMPLATES = (4, 8, 12, 16, 20, 24, 28, 30, 32)


def ksteps_of(ld16):
    ks = ld16 // 32
    return next(t for t in KSTEPS_TEMPLATES if ks <= t)


def admitted_splits(n, ld16):
    """Split sizes launch_tile_path admits: a multiple of 64 points, with a
    split's rows addressable by 31-bit byte offsets; one split up to many."""
    tiles = (n + 63) // 64
    max_tiles = ((1 << 31) - 1) // (ld16 * 2 * 64)
    out = set()
    for ns in (1, 2, 3, 5, 8, 37, 256):
        per = (tiles + ns - 1) // ns
        if per > max_tiles:
            per = max_tiles
        out.add(per * 64)
    return sorted(out)


def check_stage_loads(n, ld16, split_pts):
    """Every (split, tile, stage, wave, instruction, lane) of the X16 stage
    loads: global byte range and LDS byte range."""
    NC = (ksteps_of(ld16) * 32 + KKS - 1) // KKS
    rowbytes = ld16 * 2
    x16_bytes = n * rowbytes
    nsplit = (n + split_pts - 1) // split_pts
    lane = np.arange(KWAVE)[None, None, :]
    wave = np.arange(KTWAVES)[:, None, None]
    j = np.arange(KDMA_PER_WAVE)[None, :, None]
    inst = wave + KTWAVES * j
    # the kernel's form: instruction 0's row and k unit, rows 16 j further on
    drow0 = KROWS_PER_INST * wave + lane // KUNITS
    drow = drow0 + 16 * j
    dk = ((lane % KUNITS) ^ (drow0 & 15)) * 8
    # ... which is the swizzle of every instruction's own row
    assert (drow == KROWS_PER_INST * inst + lane // KUNITS).all()
    assert (dk == ((lane % KUNITS) ^ (drow & 15)) * 8).all()
    lds_hi = 0
    # interior splits are full splits shifted by whole splits: the first two
    # and the last two bound every one of them
    for split in sorted({0, 1, nsplit - 2, nsplit - 1} & set(range(nsplit))):
        pb = split * split_pts
        npts = split_pts if pb + split_pts < n else n - pb
        assert npts > 0
        ntile = (npts + KTP - 1) // KTP
        assert split_pts * rowbytes < (1 << 31)        # 32-bit per-lane offsets
        tiles = range(ntile) if ntile <= 64 else list(range(4)) + list(range(ntile - 4, ntile))
        for it in tiles:
            r = it * KTP + drow
            trow = np.where(r < npts, r, 0) * rowbytes
            for ic in range(NC):
                k = ic * KKS + dk
                koff = np.where(k < ld16, 2 * k, 0)
                off = pb * rowbytes + trow + koff      # bytes from X16's base
                assert off.min() >= 0
                assert (off + 16).max() <= x16_bytes, (n, ld16, split_pts, split, it, ic)
                assert ((trow + koff) < (1 << 32)).all()
                buf = (it * NC + ic) % KNBUF
                lds = buf * KSTAGE + inst * 1024 + lane * 16
                assert lds.min() >= 0 and (lds + 16).max() <= KNBUF * KSTAGE
                lds_hi = max(lds_hi, int((lds + 16).max()))
    return lds_hi


def check_epilogue_loads(n, nq, cw, split_pts):
    """Candidate words (16 B per lane), norms (4 B per lane) and bound rows
    (16 B per lane) of every tile of every (query block, split); the bound
    rows are [nq][4] words."""
    nqw = (nq + 31) // 32
    nchunk = (nqw + cw - 1) // cw
    vis_words = nchunk * n * cw
    nsplit = (n + split_pts - 1) // split_pts
    nqb = (nq + KTQ - 1) // KTQ
    lane = np.arange(KWAVE)
    for qblk in range(nqb):
        qc, wo = (4 * qblk) // cw, (4 * qblk) % cw
        assert wo + 4 <= cw
        for w in (2, 3):
            qq = qblk * KTQ + (w - 2) * KWAVE + lane
            g = KBOUND_WORDS * np.where(qq < nq, qq, 0)      # words from gthr's base
            assert g.min() >= 0 and (g + KBOUND_WORDS).max() <= KBOUND_WORDS * nq
            assert (g % 4 == 0).all()                        # 16-byte aligned
            for u in range(KEPI_BUFS):
                lds = 4 * KEPI_WORDS * u + 4 * (KEPI_THR + KBOUND_WORDS * (w - 2) * KWAVE) + 16 * lane
                assert lds.min() >= 4 * KEPI_WORDS * u + 4 * KEPI_THR
                assert (lds + 16).max() <= 4 * KEPI_WORDS * (u + 1)
        for split in sorted({0, 1, nsplit - 2, nsplit - 1} & set(range(nsplit))):
            pb = split * split_pts
            npts = split_pts if pb + split_pts < n else n - pb
            ntile = (npts + KTP - 1) // KTP
            for t in (0, ntile - 1):
                xl = t * KTP + lane
                xc = np.where(xl < npts, xl, 0)
                vis = (qc * n + pb + xc) * cw + wo          # words from visT's base
                assert vis.min() >= 0 and (vis + 4).max() <= vis_words
                e0 = 4 * KEPI_WORDS * (t & 1)              # this tile's area
                assert (e0 + 4 * KEPI_VIS + 16 * lane + 16).max() <= e0 + 4 * KEPI_NORM
                nrm = pb + xc
                assert nrm.max() < n
                assert (e0 + 4 * KEPI_NORM + 4 * lane + 4).max() <= e0 + 4 * KEPI_THR
                assert e0 + 4 * KEPI_WORDS <= KEPI_BUFS * 4 * KEPI_WORDS


def test_static_lds_allocation_is_134_5_kib():
    assert LDS_BYTES == 3 * 32768 + 2 * 3328 + 32768
    assert LDS_BYTES <= 160 * 1024


def test_pair_swap_stays_inside_the_exchange_area():
    """Wave w writes its other group's partial sums of block b at f4 slot
    (4 w + b) 64 + lane and reads its partner's (w ^ 4) slot, 16 KiB away."""
    lane = np.arange(KWAVE)
    seen = np.zeros(KTWAVES * 4 * KWAVE, dtype=int)
    for w in range(KTWAVES):
        half = w >> 2
        xdelta = -4 * 4 * KWAVE if half else 4 * 4 * KWAVE
        for b in range(4):
            wr = (4 * w + b) * KWAVE + lane
            rd = wr + xdelta
            assert wr.min() >= 0 and wr.max() < KTWAVES * 4 * KWAVE
            assert (rd == (4 * (w ^ 4) + b) * KWAVE + lane).all()
            seen[wr] += 1
    assert (seen == 1).all()          # every slot has exactly one writer


def test_b_operand_reads_are_the_swizzled_units():
    """The kernel reads k step j of wave half h at two lane offsets plus
    128 (j >> 1) elements; that is row col, unit (4 (2 j + h) + quarter) ^ col."""
    for half in (0, 1):
        for lane in range(KWAVE):
            quarter, col = lane >> 4, lane & 15
            lsel0 = col * KKS + 8 * ((4 * half + quarter) ^ (col & 7)) + 64 * (col >> 3)
            lsel1 = col * KKS + 8 * ((4 * half + quarter) ^ (col & 7)) + 64 * (1 - (col >> 3))
            for j in range(4):
                got = (lsel1 if j & 1 else lsel0) + 128 * (j >> 1)
                want = col * KKS + (((4 * (2 * j + half) + quarter) ^ col) * 8)
                assert got == want
                assert 0 <= got and got + 8 + 16 * KKS * 3 <= KSTAGE // 2


@pytest.mark.parametrize("ld16", list(range(32, 1025, 32)))
def test_stage_loads_stay_inside_x16_and_the_stages(ld16):
    for n in (1, 63, 64, 65, 1000, 4097, 60_000, 1_000_000):
        for split_pts in admitted_splits(n, ld16):
            hi = check_stage_loads(n, ld16, split_pts)
            assert hi <= KNBUF * KSTAGE


@pytest.mark.parametrize("cw", [4, 8, 16, 32])
def test_epilogue_loads_stay_inside_their_buffers(cw):
    for n in (1, 65, 4097, 60_000):
        for nq in (1, 127, 128, 129, 1000, 16_384):
            nqw = (nq + 31) // 32
            if cw > 4 and cw > 2 * nqw and cw != 32:
                continue                                  # the plan picks the smallest cw >= words
            for split_pts in admitted_splits(n, 960):
                check_epilogue_loads(n, nq, cw, split_pts)
