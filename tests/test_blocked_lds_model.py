"""CPU model of the LDS-staged sub-blocked kernel's address arithmetic
(paper_1304_7053_amd/csrc/gemm_blocked.h, gemm_blocked_lds_kernel and
blocked_lds_plan): for every size the kernel can take (the host's forced
mode, a superset of its automatic choice), both element sizes, every op
pair, padded leading dimensions and every element-aligned offset of the
matrix within its first 16 bytes:
  * every global load is a 16-byte chunk aligned to 16 bytes that overlaps
    its column (so it lies in a page the column occupies: no load can fault);
  * every LDS write stays inside the column's region of the image and inside
    the dynamic LDS the host allocates, and no LDS chunk is written twice;
  * every element the tile routine reads from the image (the element (i, j)
    at offset + i s + j pitch) was written from exactly that element's
    global bytes.
The model restates the host's plan and the kernel's chunk list."""
import itertools

import numpy as np

MAX_BYTES = 96 * 1024
THREADS, CH = 256, 6


def pitch(rows, s):
    p = ((rows * s + 30) // 16) * 16
    if (p // 16) % 2 == 0:
        p += 16
    return p


def plan(m, n, k, lda, ldb, at, bt, s, forced=True):
    """(rowsA, colsA, rowsB, colsB, pitchA, pitchB, offB, bytes) or None."""
    if m > 64 or n > 64 or k > 64 or k < 1:
        return None
    if (lda * s) % 16 or (ldb * s) % 16:
        return None
    if not forced:
        mx = max(m, n, k)
        if m <= 16 or n <= 16:
            return None
        if not at and mx < (48 if s == 4 else 32):
            return None
        if at and mx < 32:
            return None
    rA, cA = (k, m) if at else (m, k)
    rB, cB = (n, k) if bt else (k, n)
    pA, pB = pitch(rA, s), pitch(rB, s)
    offB = cA * pA
    total = offB + cB * pB
    return None if total > MAX_BYTES else (rA, cA, rB, cB, pA, pB, offB, total)


def check(m, n, k, at, bt, s, padA, padB, offA, offB_g):
    rA, cA = (k, m) if at else (m, k)
    rB, cB = (n, k) if bt else (k, n)
    lda, ldb = rA + padA, rB + padB
    pl = plan(m, n, k, lda, ldb, at, bt, s)
    if pl is None:
        return False
    rA, cA, rB, cB, pA, pB, offB, total = pl
    # global byte addresses relative to a 16-aligned origin per operand
    ga, gb = offA, (1 << 20) + offB_g
    a16, b16 = ga & ~15, gb & ~15
    nqA = ((ga & 15) + rA * s + 15) >> 4
    nqB = ((gb & 15) + rB * s + 15) >> 4
    totA, totB = cA * nqA, cB * nqB
    passes = -(-max(totA, totB) // (THREADS * CH))
    # the kernel's per-thread walk: (column, chunk) starts at divmod(t, nq) and
    # advances by the constant step 256 = dj nq + dq with one carry
    srcs, dsts = [], []
    for name, tot, nq, o16, ld, img, pit, base in (("A", totA, nqA, a16, lda * s, 0, pA, ga),
                                                   ("B", totB, nqB, b16, ldb * s, offB, pB, gb)):
        t = np.arange(THREADS)
        j, q = t // nq, t % nq
        dj, dq = THREADS // nq, THREADS % nq
        for c in range(passes * CH):
            idx = c * THREADS + t           # slot c of every thread, in pass order
            assert np.array_equal(j * nq + q, idx)
            ok = idx < tot
            src = np.where(ok, o16 + j * ld + 16 * q, o16)
            dst = np.where(ok, img + j * pit + 16 * q, -1)
            lo = np.where(ok, base + j * ld, base)
            hi = lo + np.where(ok, (rA if name == "A" else rB) * s, s)
            assert np.all(src % 16 == 0)
            assert np.all(src < hi) and np.all(src + 16 > lo), (name, m, n, k, at, bt, s)
            w = ok
            assert np.all(dst[w] >= img + j[w] * pit) and np.all(dst[w] + 16 <= img + (j[w] + 1) * pit)
            srcs.append(src[w])
            dsts.append(dst[w])
            q = q + dq
            j = j + dj
            carry = q >= nq
            q = np.where(carry, q - nq, q)
            j = np.where(carry, j + 1, j)
    src = np.concatenate(srcs)
    dst = np.concatenate(dsts)
    assert len(dst) == totA + totB                 # every chunk of both lists, once
    assert np.all(dst + 16 <= total)
    assert len(np.unique(dst)) == len(dst)
    # element (i, j) of each image: its LDS bytes come from its global bytes
    lds_src = dict(zip(dst.tolist(), src.tolist()))
    for (rows, cols, base, ld, img0, pit) in ((rA, cA, ga, lda, 0, pA), (rB, cB, gb, ldb, offB, pB)):
        for jj in sorted({0, cols // 2, cols - 1}):
            for ii in sorted({0, rows // 2, rows - 1}):
                lpos = img0 + (base & 15) + ii * s + jj * pit
                gpos = base + ii * s + jj * ld * s
                chunk = lpos & ~15
                assert chunk in lds_src, (rows, cols, ii, jj)
                assert lds_src[chunk] + (lpos - chunk) == gpos
                assert lpos + s <= chunk + 16
    return True


def test_lds_blocked_accesses_every_routed_shape():
    sizes = [1, 5, 16, 17, 20, 24, 31, 32, 33, 40, 48, 57, 63, 64]
    ran = 0
    for s in (4, 8):
        offs = range(0, 16, s)
        for m, n, k in itertools.product(sizes, sizes, sizes):
            if max(m, n, k) <= 16 or (m * 7 + n * 3 + k) % 5:
                continue                         # a fifth of the shapes
            for at, bt in itertools.product((False, True), (False, True)):
                for padA, padB in ((0, 0), (16 // s * 3, 16 // s)):
                    rA = k if at else m
                    rB = n if bt else k
                    if ((rA + padA) * s) % 16 or ((rB + padB) * s) % 16:
                        continue
                    for oa in offs:
                        ran += check(m, n, k, at, bt, s, padA, padB, oa, (oa + 4 * s) % 16)
    assert ran > 500


def test_plan_rejects_what_the_kernel_cannot_take():
    assert plan(65, 20, 20, 68, 20, False, False, 4) is None          # above 64
    assert plan(20, 20, 0, 20, 1, False, False, 4) is None            # k = 0
    assert plan(21, 20, 20, 21, 20, False, False, 4) is None          # lda * 4 not a multiple of 16
    assert plan(64, 64, 64, 64, 64, False, False, 8) is not None      # f64 n = 64: 2 x 64 x 528 bytes
    assert plan(64, 64, 64, 64 * 3, 64, False, False, 8) is not None  # padding does not change the image
    # the automatic choice: reuse of A and B from size 32 on; 4-byte types with op(A) N from 48
    assert plan(24, 24, 24, 24, 24, False, False, 4, forced=False) is None
    assert plan(32, 32, 32, 32, 32, True, False, 4, forced=False) is not None
    assert plan(32, 32, 32, 32, 32, False, False, 4, forced=False) is None
    assert plan(32, 32, 32, 32, 32, False, False, 8, forced=False) is not None
    assert plan(48, 48, 48, 48, 48, False, False, 4, forced=False) is not None
    assert plan(64, 16, 64, 64, 64, False, False, 4, forced=False) is None
    assert pitch(64, 4) == 272 and pitch(64, 8) == 528 and pitch(32, 4) == 144
