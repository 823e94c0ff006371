"""CPU model of how the e4m3 quantiser (paper_1304_7053_amd/csrc/quant.hip)
stores a column of codes: up to 3 head bytes to the first 4-byte boundary,
whole aligned dwords built by a byte funnel shift of the four code words,
then up to 3 tail bytes.  For every start address modulo 4 and every row
count 0..16: every byte of [start, start + rows) is written exactly once
with its code, nothing outside it is written, and every dword store is
4-byte aligned."""
import numpy as np


def alignbyte(hi, lo, s):
    """Bytes s .. s+3 of the 8-byte value hi:lo (s in 0..3)."""
    return ((((hi & 0xFFFFFFFF) << 32) | (lo & 0xFFFFFFFF)) >> (8 * (s & 3))) & 0xFFFFFFFF


def store_plan(addr, rows, codes):
    """(address, byte) pairs the kernel writes for one column."""
    out = []
    h0 = (-addr) & 3
    h = min(h0, rows)
    nd = (rows - h) >> 2
    tb = h + 4 * nd
    for j in range(3):
        if j < h:
            out.append((addr + j, (codes[0] >> (8 * j)) & 0xFF))
    for i in range(4):
        if i < nd:
            a = addr + h + 4 * i
            assert a % 4 == 0
            w = alignbyte(codes[i + 1] if i < 3 else 0, codes[i], h)
            out += [(a + b, (w >> (8 * b)) & 0xFF) for b in range(4)]
    for j in range(3):
        e = tb + j
        w = codes[min(e >> 2, 3)]
        if e < rows:
            out.append((addr + e, (w >> (8 * (e & 3))) & 0xFF))
    return out


def test_every_alignment_and_row_count():
    g = np.random.default_rng(5)
    for base in (4096, 4096 + 64):
        for a in range(4):
            for rows in range(17):
                byts = g.integers(0, 256, size=16)
                codes = [int(byts[4 * d] | (byts[4 * d + 1] << 8) | (byts[4 * d + 2] << 16) | (byts[4 * d + 3] << 24))
                         for d in range(4)]
                addr = base + a
                w = store_plan(addr, rows, codes)
                addrs = [x for x, _ in w]
                assert sorted(addrs) == list(range(addr, addr + rows)), (a, rows)
                for x, v in w:
                    assert v == byts[x - addr], (a, rows, x - addr)
                assert len(w) <= 16 and sum(1 for _ in w) == rows
