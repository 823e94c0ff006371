"""CPU model of the LDS-staged kernel's address arithmetic
(paper_1304_7053_amd/csrc/gemm_staged.h): every global load and store, every
LDS write and read of every lane stays inside its span, its allocation and
its LDS region, for every size 1..16 and the run lengths the host picks.

The model restates the host's run-length choice (staged_run_length,
staged_whole_chunks) and the kernel's chunk lists (general path: whole
chunks plus one overlapping tail per span; slot-table path for runs of whole
chunks) and checks the accesses of the first, the last full and the last
(shorter) run; every other run has the same offsets relative to its spans.
It guards the case that once faulted: alpha = beta = 0, where a run has no
chunk to load and the slot table must still read inside the C span."""
import itertools

import numpy as np
import pytest

LANES = 64


def size_class(m, n, k):
    mx = max(m, n, k)
    return 4 if mx <= 4 else (8 if mx <= 8 else 16)


def lds_bytes_per_wave(ec):
    return 16384 if ec >= 16 else 8192


def staged_run_length(m, n, k, batch, min_waves, ei, ec):
    """The host's choice of matrices per run (0: the staged kernel does not apply)."""
    if m < 1 or n < 1 or k < 1 or batch < 1:
        return 0
    per = (m * k + k * n) * ei + m * n * ec
    room = lds_bytes_per_wave(ec) - 32
    if per > room:
        return 0
    G = min(room // per, 256)
    fair = (batch + min_waves - 1) // min_waves
    if fair < G:
        G = max(fair, 1)
    P = 16 // size_class(m, n, k)
    step = 4 if (ei < 4 and P < 4) else P

    def whole16(b):
        low = b & -b
        return 16 // (low if low < 16 else 16)

    unit = step
    for b in (m * k * ei, k * n * ei, m * n * ec):
        unit = max(unit, whole16(b))
    if G >= unit:
        G -= G % unit
    elif unit * per <= room:
        G = unit
    elif G >= step:
        G -= G % step
    elif step * per <= room:
        G = step
    G = min(G, batch)
    last = batch - ((batch - 1) // G) * G
    for c in (G, last):
        if c * m * k * ei < 16 or c * k * n * ei < 16 or c * m * n * ec < 16:
            return 0
        if (c * m * k * ei) % 4 or (c * k * n * ei) % 4:
            return 0
    return G


def whole_chunks(m, n, k, G, ei, ec):
    return (G * m * k * ei) % 16 == 0 and (G * k * n * ei) % 16 == 0 and (G * m * n * ec) % 16 == 0


class Checker:
    """Records accesses as (space, lo, hi) byte ranges and checks them."""

    def __init__(self, alloc, regions, ldsw):
        self.alloc = alloc          # {"A": bytes, ...}
        self.regions = regions      # {"A": (lo, hi), ...} in the wave's LDS slice
        self.ldsw = ldsw

    def glob(self, op, lo, span):
        """16-byte global access at byte lo of operand op, inside span (lo_s, hi_s)."""
        lo = np.atleast_1d(np.asarray(lo, dtype=np.int64))
        assert np.all(lo >= span[0]) and np.all(lo + 16 <= span[1]), (op, lo.min(), lo.max(), span)
        assert span[0] >= 0 and span[1] <= self.alloc[op], (op, span, self.alloc[op])

    def lds(self, op, lo, size=16):
        lo = np.atleast_1d(np.asarray(lo, dtype=np.int64))
        r = self.regions[op]
        assert np.all(lo >= r[0]) and np.all(lo + size <= r[1]), (op, lo.min(), lo.max(), r)
        assert r[1] <= self.ldsw


def run_spans(r, G, batch, eA, eB, eC, ei, ec, a0, b0):
    p0 = r * G
    cnt = min(batch - p0, G)
    base = {"A": p0 * eA * ei, "B": p0 * eB * ei, "C": p0 * eC * ec}
    S = {"A": 0 if a0 else cnt * eA * ei, "B": 0 if a0 else cnt * eB * ei}
    SC = cnt * eC * ec
    S["Cin"] = 0 if b0 else SC
    return cnt, base, S, SC


def check_general_run(ck, r, G, batch, dims, ei, ec, a0, b0, offB, offC, maxch):
    m, n, k = dims
    eA, eB, eC = m * k, k * n, m * n
    cnt, base, S, SC = run_spans(r, G, batch, eA, eB, eC, ei, ec, a0, b0)
    FA, FB, FC_in = S["A"] >> 4, S["B"] >> 4, S["Cin"] >> 4
    FT = FA + FB + FC_in
    assert (FT + 63) // 64 <= maxch, "chunk list longer than the lane slots"
    q = np.arange(FT)
    inA, inB = q < FA, (q >= FA) & (q < FA + FB)
    off = 16 * np.where(inA, q, np.where(inB, q - FA, q - FA - FB))
    for op, sel, dst0, span_len in (("A", inA, 0, S["A"]), ("B", inB, offB, S["B"]),
                                    ("C", ~inA & ~inB, offC, S["Cin"])):
        if sel.any():
            ck.glob(op, base[op] + off[sel], (base[op], base[op] + span_len))
            ck.lds(op, dst0 + off[sel])
    # tails (lanes 0..2); without a tail the lane re-reads the head of the C span
    for j, (op, S_, dst0) in enumerate((("A", S["A"], 0), ("B", S["B"], offB), ("C", S["Cin"], offC))):
        has = (S_ & 15) != 0
        if has:
            ck.glob(op, base[op] + S_ - 16, (base[op], base[op] + S_))
            ck.lds(op, dst0 + S_ - 16)
        else:
            ck.glob("C", base["C"], (base["C"], base["C"] + SC))
    # compute: lane tiles read matrices mi < cnt (lanes past the run: cnt - 1)
    mi = np.arange(cnt)
    ck.lds("A", mi * eA * ei, eA * ei)
    ck.lds("B", offB + mi * eB * ei, eB * ei)
    ck.lds("C", offC + mi * eC * ec, eC * ec)
    # store: whole C chunks, then the overlapping tail
    FC = SC >> 4
    assert (FC + 63) // 64 <= maxch
    qc = np.arange(FC)
    if FC:
        ck.lds("C", offC + 16 * qc)
        ck.glob("C", base["C"] + 16 * qc, (base["C"], base["C"] + SC))
    if SC & 15:
        ck.lds("C", offC + SC - 16)
        ck.glob("C", base["C"] + SC - 16, (base["C"], base["C"] + SC))
    return cnt


def check_fast_runs(ck, G, batch, dims, ei, ec, a0, b0, offB, offC, maxch):
    """Slot-table path: every slot loads on every full run."""
    m, n, k = dims
    eA, eB, eC = m * k, k * n, m * n
    fSA = 0 if a0 else G * eA * ei
    fSB = 0 if a0 else G * eB * ei
    fSC = G * eC * ec
    fSCin = 0 if b0 else fSC
    fFA, fFB = fSA >> 4, fSB >> 4
    fFT = fFA + fFB + (fSCin >> 4)
    fNT = (fFT + 63) >> 6
    fFC = fSC >> 4
    fNC = (fFC + 63) >> 6
    assert fNT <= maxch and fNC <= maxch
    lane = np.arange(LANES)[:, None]
    t = np.arange(maxch)[None, :]
    q = lane + 64 * t
    q = np.where(q < fFT, q, fFT - 1 if fFT > 0 else 0)
    j = np.where(q < fFA, 0, np.where(q < fFA + fFB, 1, 2))
    off = 16 * np.where(j == 0, q, np.where(j == 1, q - fFA, q - fFA - fFB))
    dst = np.where(j == 0, 0, np.where(j == 1, offB, offC)) + off
    assert off.max() < (1 << 14) and dst.max() < (1 << 14), "slot fields overflow 14 bits"
    nfull = batch // G
    for r in sorted({0, max(nfull - 1, 0)}):
        if r >= nfull:
            continue
        span = {"A": (r * G * eA * ei, r * G * eA * ei + fSA), "B": (r * G * eB * ei, r * G * eB * ei + fSB),
                "C": (r * G * eC * ec, r * G * eC * ec + fSC)}
        for jj, op in enumerate("ABC"):
            sel = j == jj
            if sel.any():
                # a C slot reads inside the run's C span even when C is not an input
                ck.glob(op, span[op][0] + off[sel], span[op])
        written = np.broadcast_to(t < fNT, j.shape)
        for jj, op in enumerate("ABC"):
            sel = (j == jj) & written
            if sel.any():
                ck.lds(op, dst[sel])
        mi = np.arange(G)
        ck.lds("A", mi * eA * ei, eA * ei)
        ck.lds("B", offB + mi * eB * ei, eB * ei)
        ck.lds("C", offC + mi * eC * ec, eC * ec)
        qc = lane + 64 * t
        qc = np.where(qc < fFC, qc, fFC - 1)[t.repeat(LANES, 0) < fNC]
        ck.lds("C", offC + 16 * qc)
        ck.glob("C", span["C"][0] + 16 * qc, span["C"])
    return nfull


TYPES = {"s": (4, 4), "d": (8, 8), "c": (8, 8), "z": (16, 16), "bf16": (2, 4)}


def check_config(ei, ec, m, n, k, batch, a0, b0, min_waves):
    G = staged_run_length(m, n, k, batch, min_waves, ei, ec)
    if G == 0:
        return False
    eA, eB, eC = m * k, k * n, m * n
    ldsw = lds_bytes_per_wave(ec)
    maxch = ldsw // 1024
    offB = (G * eA * ei + 15) & ~15
    offC = offB + ((G * eB * ei + 15) & ~15)
    regions = {"A": (0, G * eA * ei), "B": (offB, offB + G * eB * ei), "C": (offC, offC + G * eC * ec)}
    alloc = {"A": batch * eA * ei, "B": batch * eB * ei, "C": batch * eC * ec}
    ck = Checker(alloc, regions, ldsw)
    nruns = (batch + G - 1) // G
    if whole_chunks(m, n, k, G, ei, ec):
        nfull = check_fast_runs(ck, G, batch, (m, n, k), ei, ec, a0, b0, offB, offC, maxch)
        if nfull < nruns:
            check_general_run(ck, nfull, G, batch, (m, n, k), ei, ec, a0, b0, offB, offC, maxch)
    else:
        for r in sorted({0, max(nruns - 2, 0), nruns - 1}):
            check_general_run(ck, r, G, batch, (m, n, k), ei, ec, a0, b0, offB, offC, maxch)
    return True


@pytest.mark.parametrize("prefix", list(TYPES))
def test_staged_accesses_in_bounds_every_size(prefix):
    ei, ec = TYPES[prefix]
    sizes = range(1, 17)
    # (batch, waves the host keeps busy): a single matrix, a short batch,
    # a batch whose last run is short, and few waves (long runs)
    cases = ((1, 4096), (17, 4096), (100_003, 4096), (1000, 64)) if prefix == "s" else ((17, 4096), (100_003, 4096))
    scal = list(itertools.product((False, True), (False, True)))
    ran = 0
    for m, n, k in itertools.product(sizes, sizes, sizes):
        if prefix != "s" and (m + n + k) % 3:
            continue                                       # a third of the shapes for the other types
        for batch, mw in cases:
            for a0, b0 in scal:
                ran += check_config(ei, ec, m, n, k, batch, a0, b0, mw)
    assert ran > 1000


def test_model_rejects_a_planted_overrun():
    """The checker itself: a tail taken from a span shorter than 16 bytes
    (what the run-length rule excludes) is reported."""
    ck = Checker({"A": 64}, {"A": (0, 64)}, 8192)
    with pytest.raises(AssertionError):
        ck.glob("A", 12 - 16, (0, 12))
    with pytest.raises(AssertionError):
        ck.lds("A", 56)
