"""Host check of the LDS layout of the BF16, x10 and INT8 products against
the bank model measured on gfx950 (probe kernels reading and writing 16-byte
LDS vectors at per-lane address tables, counted by SQ_LDS_IDX_ACTIVE and
SQ_LDS_BANK_CONFLICT): ds_read_b128 serves a wave in four passes of 16 lanes
over 256 bytes of banks, a pass taking the lane quads {0,3,5,6}, {1,2,4,7},
{8,11,13,14} or {9,10,12,15} (quad j = lanes 4j..4j+3); ds_write_b128 in
eight passes of 8 consecutive lanes over 128 bytes.  Rows are 64 bytes (four
16-byte chunks); chunk c of row r sits at c ^ f(r), f(r) = (r / 2) mod 4.
A pass is conflict-free when its lanes touch distinct 16-byte bank slots."""
import re
from pathlib import Path

CSRC = Path(__file__).resolve().parents[1] / "paper_2512_13550_amd" / "csrc"
READ_PASSES = [[4 * q + i for q in quads for i in range(4)]
               for quads in ((0, 3, 5, 6), (1, 2, 4, 7), (8, 11, 13, 14), (9, 10, 12, 15))]
WRITE_PASSES = [list(range(8 * p, 8 * p + 8)) for p in range(8)]


def f(r):
    return (r >> 1) & 3


def addr(r, c):
    return r * 64 + 16 * (c ^ f(r))


def conflict_free(lane_addr, passes, span):
    for lanes in passes:
        slots = [(lane_addr(l) % span) // 16 for l in lanes]
        if len(set(slots)) != len(slots):
            return False
    return True


def test_kernels_use_this_swizzle():
    """The three product sources place chunk c of row r at c ^ ((r >> 1) & 3)."""
    for name, fn in (("gemm_fx.hip", "swz"), ("gemm_bf16.hip", "swz"), ("gemm_i8.hip", "swz16")):
        src = (CSRC / name).read_text()
        m = re.search(r"int %s\(int r, int c\) \{ return \(c \^ \(\(r >> 1\) & 3\)\) << \d; \}" % fn, src)
        assert m, name


def test_fragment_reads_conflict_free():
    """Lane l reads chunk l / 16 of row R + l % 16, R a multiple of 16."""
    for R in range(0, 256, 16):
        assert conflict_free(lambda l: addr(R + (l & 15), l >> 4), READ_PASSES, 256), R


def test_kmajor_and_row_writes_conflict_free():
    """Column loader: lane l writes one chunk of row R + l (R a multiple of
    64); row loader: four lanes write the four chunks of one row."""
    for R in range(0, 256, 64):
        for c in range(4):
            assert conflict_free(lambda l: addr(R + l, c), WRITE_PASSES, 128), (R, c)
    for R in range(0, 256, 16):
        assert conflict_free(lambda l: addr(R + (l >> 2), l & 3), WRITE_PASSES, 128), R


def test_previous_swizzle_conflicts_under_the_model():
    """The swizzle built for consecutive-lane passes, c ^ (((r >> 2) & 3) ^
    (r & 2)), puts two lanes of every read pass on one slot: what the
    counter showed (0.37-0.44 of the LDS cycles) before the change."""
    old = lambda r, c: r * 64 + 16 * (c ^ (((r >> 2) & 3) ^ (r & 2)))
    assert not conflict_free(lambda l: old(l & 15, l >> 4), READ_PASSES, 256)
