"""GPU parity of the precision modes (binary32 accumulation and C): bf16,
fp16 and fp8-e4m3 inputs (with per-matrix absmax scales produced by the
library's quantiser) and the BF16x3 split mode.

Kernel-only parity: the oracle evaluates the same stored (decoded, scaled)
operands exactly, so products of narrow values being exact in binary32 the
bound is the plain 4 max(k,1) u, u = 2^-24.  BF16x3 accumulates three
products per k-step: its bound is 4 * 3 max(k,1) u against the oracle's
split product.  The error of each mode against the binary32-input product
(the quantisation error) is reported, not pinned."""
import numpy as np
import pytest
import torch

import oracle
from paper_1304_7053_amd import inputs, sbg
from gpu_util import VarCase, check_var, from_dev, normalised_error, say, to_dev

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
NARROW = {"bf16": (torch.bfloat16, sbg.R_16BF), "f16": (torch.float16, sbg.R_16F)}


def strided_inputs(g, ta, tb, m, n, k, batch, dist="uniform"):
    ra, ca = (m, k) if ta == "N" else (k, m)
    rb, cb = (k, n) if tb == "N" else (n, k)
    A = inputs.strided_batch(g, batch, ra, ca, ra, ra * ca, np.float32, dist)
    B = inputs.strided_batch(g, batch, rb, cb, rb, rb * cb, np.float32, dist)
    C = inputs.strided_batch(g, batch, m, n, m, m * n, np.float32, dist)
    return A, B, C, ra, rb


def unpack(flat, batch, m, n):
    return np.swapaxes(flat.reshape(batch, n, m), 1, 2)


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
@pytest.mark.parametrize("dist", ["uniform", "logu"])
def test_half_inputs_strided(gpu_lib, fmt, dist):
    tdt, code = NARROW[fmt]
    g = inputs.rng(4, salt=10)
    for (ta, tb, s) in [("N", "N", 16), ("T", "N", 8), ("N", "T", 5), ("T", "T", 13), ("N", "N", 1)]:
        batch = 1001
        A, B, C, ra, rb = strided_inputs(g, ta, tb, s, s, s, batch, dist)
        dA = torch.from_numpy(A).to("cuda").to(tdt)
        dB = torch.from_numpy(B).to("cuda").to(tdt)
        dC = to_dev(C)
        say(f"{fmt} {dist} {ta}{tb} n={s}")
        sbg.gemm_strided_ex(ta, tb, s, s, s, 1.5, dA, ra, ra * s, None, dB, rb, rb * s, None, -0.5, dC, s, s * s,
                            batch, code)
        torch.cuda.synchronize()
        Ab = dA.view(torch.int16).cpu().numpy().view(np.uint16)
        Bb = dB.view(torch.int16).cpu().numpy().view(np.uint16)
        types = (fmt, fmt, "f32")
        hi, lo = oracle.gemm_strided(ta, tb, s, s, s, 1.5, Ab, ra, ra * s, Bb, rb, rb * s, -0.5, C, s, s * s,
                                     batch, ext=True, types=types)
        bnd = oracle.bound_strided(ta, tb, s, s, s, 1.5, Ab, ra, ra * s, Bb, rb, rb * s, -0.5, C, s, s * s, batch,
                                   types=types)
        got = unpack(from_dev(dC), batch, s, s)
        e = normalised_error(got, hi, lo, bnd)
        assert np.max(e) <= 4 * max(s, 1) * U32, (fmt, ta, tb, s, np.max(e) / U32)
        # end-to-end error against the binary32 inputs (reported)
        h32, l32 = oracle.gemm_strided(ta, tb, s, s, s, 1.5, A, ra, ra * s, B, rb, rb * s, -0.5, C, s, s * s,
                                       batch, ext=True)
        b32 = oracle.bound_strided(ta, tb, s, s, s, 1.5, A, ra, ra * s, B, rb, rb * s, -0.5, C, s, s * s, batch)
        say(f"  end-to-end max normalised error vs fp32 inputs: {np.max(normalised_error(got, h32, l32, b32)):.3e}")


def test_quantiser_matches_oracle_bitwise(gpu_lib):
    g = inputs.rng(4, salt=11)
    for (rows, cols, dist) in [(16, 16, "uniform"), (7, 3, "logu"), (1, 1, "uniform"), (12, 9, "logu")]:
        batch, ld = 777, rows + 2
        X = inputs.strided_batch(g, batch, rows, cols, ld, ld * cols + 1, np.float32, dist, fill=np.nan)
        X[: ld * cols + 1][np.isfinite(X[: ld * cols + 1])] = 0.0        # an all-zero matrix: scale 1
        dX = to_dev(X)
        dQ = torch.full((batch * rows * cols + 5,), 0xAB, dtype=torch.uint8, device="cuda")
        dS = torch.zeros(batch, dtype=torch.float32, device="cuda")
        say(f"quantise {rows}x{cols} {dist}")
        sbg.quantize_e4m3_strided(rows, cols, dX, ld, ld * cols + 1, dQ, rows, rows * cols, dS, batch)
        torch.cuda.synchronize()
        off = np.arange(batch, dtype=np.int64) * (ld * cols + 1)
        Q, offQ, S = oracle.quant_e4m3(X, off, rows, cols, ld, batch)
        assert np.array_equal(from_dev(dS), S)
        assert np.array_equal(from_dev(dQ)[: batch * rows * cols], Q[: batch * rows * cols])
        assert np.all(from_dev(dQ)[batch * rows * cols:] == 0xAB)


@pytest.mark.parametrize("dist", ["uniform", "logu"])
def test_quantiser_vbatched_matches_oracle_bitwise(gpu_lib, dist):
    """Variable-size quantiser: sizes 0..16 drawn per matrix, padded leading
    dimensions on both sides (NaN in the gaps of X), an all-zero matrix, and
    two rejected matrices (rows above the bound; ldq too small), whose codes
    and scale stay untouched.  Codes and scales bit for bit against the oracle;
    the bytes between Q's columns are left alone."""
    g = inputs.rng(4, salt=12 if dist == "uniform" else 13)
    N = 2001
    rows = g.integers(0, 17, size=N).astype(np.int32)
    cols = g.integers(0, 17, size=N).astype(np.int32)
    rows[:3] = 16
    cols[:3] = 16
    rows[7] = max(int(rows[7]), 2)
    ldx = (np.maximum(rows, 1) + g.integers(0, 3, size=N)).astype(np.int32)
    ldq = (np.maximum(rows, 1) + g.integers(0, 2, size=N)).astype(np.int32)
    bad = np.zeros(N, dtype=bool)
    ldq[7], bad[7] = int(rows[7]) - 1, True     # leading dimension of Q too small
    sizeX = np.maximum(ldx.astype(np.int64) * cols, 1)
    sizeQ = np.maximum(ldq.astype(np.int64) * cols, 1)
    offX = np.concatenate([[0], np.cumsum(sizeX)[:-1]])
    offQ = np.concatenate([[0], np.cumsum(sizeQ)[:-1]])
    X = np.full(int(sizeX.sum()), np.nan, dtype=np.float32)
    for p in range(N):
        r, c = int(rows[p]), int(cols[p])
        if r and c:
            idx = offX[p] + np.arange(c)[:, None] * ldx[p] + np.arange(r)[None, :]
            X[idx] = inputs.DISTS[dist](g, (c, r), np.float32)
    X[offX[1] + np.arange(int(ldx[1]) * int(cols[1]))] = 0.0    # matrix 1: all zero (scale 1)
    rows_dev = rows.copy()
    rows_dev[5], bad[5] = 17, True              # above max_rows
    dX = to_dev(X)
    dQ = torch.full((int(sizeQ.sum()),), 0xAB, dtype=torch.uint8, device="cuda")
    dS = torch.full((N,), -7.0, dtype=torch.float32, device="cuda")
    pX = torch.tensor(dX.data_ptr() + offX * 4, device="cuda")
    pQ = torch.tensor(dQ.data_ptr() + offQ, device="cuda")
    say(f"quantise variable-size N={N} {dist}")
    sbg.quantize_e4m3_vbatched(torch.from_numpy(rows_dev).cuda(), torch.from_numpy(cols).cuda(), 16, 16, pX,
                               torch.from_numpy(ldx).cuda(), pQ, torch.from_numpy(ldq).cuda(), dS, N)
    torch.cuda.synchronize()
    Qg, Sg = from_dev(dQ), from_dev(dS)
    good = np.nonzero(~bad)[0]
    Qo, offO, So = oracle.quant_e4m3(X, offX[good], rows[good], cols[good], ldx[good], len(good))
    for q, p in enumerate(good):
        r, c = int(rows[p]), int(cols[p])
        got = Qg[offQ[p] + np.arange(c)[:, None] * ldq[p] + np.arange(r)[None, :]]
        ref = Qo[offO[q]:offO[q] + r * c].reshape(c, r)
        assert np.array_equal(got, ref), p
        assert Sg[p] == (So[q] if r and c else 1.0), (p, Sg[p], So[q])
    for p in np.nonzero(bad)[0]:
        assert Sg[p] == -7.0, p
        assert np.all(Qg[offQ[p]:offQ[p] + sizeQ[p]] == 0xAB), p
    # the gaps between columns (ldq > rows) keep their bytes
    mask = np.ones(Qg.size, dtype=bool)
    for p in good:
        r, c = int(rows[p]), int(cols[p])
        mask[offQ[p] + np.arange(c)[:, None] * ldq[p] + np.arange(r)[None, :]] = False
    assert np.all(Qg[mask] == 0xAB)


def test_quantiser_rounding_boundaries_full_size(gpu_lib):
    """200,000 16 x 16 matrices (the var-size workload's count at its largest
    size), codes and scales bit for bit against the oracle.  The first 3,072
    are built so that v / s falls near every e4m3 rounding boundary with
    scales 1, 3, 5, 0.75, 7 2^-20 and 3 2^40, alternating by wave: on it or up
    to 3 ulps away (ties included; the reciprocal product's bracket straddles
    the boundary and the wave divides), or 20 and 40 ulps away (the wave keeps
    the product's codes).  The rest are normal values, mostly on the
    reciprocal path."""
    g = inputs.rng(4, salt=14)
    batch, n = 200_000, 16
    X = g.standard_normal(batch * n * n).astype(np.float32)
    codes = np.arange(0x7F)
    vals = np.unique([oracle.decode(int(c), "e4m3") for c in codes])
    mids = (vals[1:] + vals[:-1]) / 2
    scs = np.array([1.0, 3.0, 5.0, 0.75, 7.0 * 2.0 ** -20, 3.0 * 2.0 ** 40], dtype=np.float32)
    K = 3072
    NEAR, FAR = np.arange(-3, 4), np.array([-40, -20, 20, 40])
    for p in range(K):
        sc = scs[p % len(scs)]
        el = np.arange(n * n - 1) + p
        v = (np.where(el % 2, -1.0, 1.0) * mids[(el // 2) % len(mids)] * np.float64(sc)).astype(np.float32)
        ulps = NEAR if (p // 4) % 2 == 0 else FAR             # 4 matrices to a wave: whole waves near or far
        k = ulps[(el // (2 * len(mids)) + p) % len(ulps)]   # ulps of magnitude away from the boundary
        v = (v.view(np.int32) + k.astype(np.int32)).view(np.float32)
        X[p * n * n] = np.float32(448.0) * sc
        X[p * n * n + 1:(p + 1) * n * n] = v
    dX = to_dev(X)
    dQ = torch.full((batch * n * n,), 0xAB, dtype=torch.uint8, device="cuda")
    dS = torch.zeros(batch, dtype=torch.float32, device="cuda")
    say(f"quantise {batch} x {n}x{n}, rounding boundaries in the first {K}")
    sbg.quantize_e4m3_strided(n, n, dX, n, n * n, dQ, n, n * n, dS, batch)
    torch.cuda.synchronize()
    Q, offQ, S = oracle.quant_e4m3(X, np.arange(batch, dtype=np.int64) * n * n, n, n, n, batch)
    assert np.array_equal(S[:K], np.resize(scs, K))       # the built matrices have the scales they were built for
    Sg, Qg = from_dev(dS), from_dev(dQ)
    assert np.array_equal(Sg, S)
    bad = np.nonzero(Qg != Q[: batch * n * n])[0]
    assert bad.size == 0, (bad.size, bad[:8], X[bad[:8]])


@pytest.mark.parametrize("dist", ["uniform", "logu"])
def test_fp8_scaled_strided(gpu_lib, dist):
    g = inputs.rng(4, salt=12)
    for (ta, tb, s) in [("N", "N", 16), ("T", "N", 8), ("N", "T", 3), ("T", "T", 11)]:
        batch = 903
        A, B, C, ra, rb = strided_inputs(g, ta, tb, s, s, s, batch, dist)
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        qA = torch.empty(A.size, dtype=torch.uint8, device="cuda")
        qB = torch.empty(B.size, dtype=torch.uint8, device="cuda")
        sA = torch.empty(batch, dtype=torch.float32, device="cuda")
        sB = torch.empty(batch, dtype=torch.float32, device="cuda")
        say(f"fp8 {dist} {ta}{tb} n={s}")
        sbg.quantize_e4m3_strided(ra, s if ta == "N" else s, dA, ra, ra * s, qA, ra, ra * s, sA, batch)
        sbg.quantize_e4m3_strided(rb, s, dB, rb, rb * s, qB, rb, rb * s, sB, batch)
        sbg.gemm_strided_ex(ta, tb, s, s, s, 1.5, qA, ra, ra * s, sA, qB, rb, rb * s, sB, -0.5, dC, s, s * s, batch,
                            sbg.R_8F_E4M3)
        torch.cuda.synchronize()
        Qa, Qb = from_dev(qA), from_dev(qB)
        Sa, Sb = from_dev(sA).astype(np.float64), from_dev(sB).astype(np.float64)
        types = ("e4m3", "e4m3", "f32")
        hi, lo = oracle.gemm_strided(ta, tb, s, s, s, 1.5, Qa, ra, ra * s, Qb, rb, rb * s, -0.5, C, s, s * s, batch,
                                     ext=True, types=types, scaleA=Sa, scaleB=Sb)
        bnd = oracle.bound_strided(ta, tb, s, s, s, 1.5, Qa, ra, ra * s, Qb, rb, rb * s, -0.5, C, s, s * s, batch,
                                   types=types, scaleA=Sa, scaleB=Sb)
        got = unpack(from_dev(dC), batch, s, s)
        e = normalised_error(got, hi, lo, bnd)
        assert np.max(e) <= 4 * max(s, 1) * U32, (ta, tb, s, np.max(e) / U32)
        h32, l32 = oracle.gemm_strided(ta, tb, s, s, s, 1.5, A, ra, ra * s, B, rb, rb * s, -0.5, C, s, s * s,
                                       batch, ext=True)
        b32 = oracle.bound_strided(ta, tb, s, s, s, 1.5, A, ra, ra * s, B, rb, rb * s, -0.5, C, s, s * s, batch)
        say(f"  end-to-end max normalised error vs fp32 inputs: {np.max(normalised_error(got, h32, l32, b32)):.3e}")


@pytest.mark.parametrize("dist", ["uniform", "logu"])
def test_bf16x3_strided(gpu_lib, dist):
    g = inputs.rng(4, salt=13)
    for (ta, tb, s) in [("N", "N", 16), ("T", "N", 9), ("N", "T", 4), ("T", "T", 16)]:
        batch = 1003
        A, B, C, ra, rb = strided_inputs(g, ta, tb, s, s, s, batch, dist)
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        say(f"bf16x3 {dist} {ta}{tb} n={s}")
        sbg.gemm_strided_ex(ta, tb, s, s, s, 1.5, dA, ra, ra * s, None, dB, rb, rb * s, None, -0.5, dC, s, s * s,
                            batch, sbg.R_32F, sbg.MODE_BF16X3)
        torch.cuda.synchronize()
        p = np.arange(batch, dtype=np.int64)
        hi, lo, bnd, _, _, _ = oracle.gemm_split3_general(ta, tb, s, s, s, 1.5, A, p * ra * s, ra, B, p * rb * s,
                                                          rb, -0.5, C, p * s * s, s, batch)
        got = unpack(from_dev(dC), batch, s, s)
        e = normalised_error(got, unpack(hi, batch, s, s), unpack(lo, batch, s, s), unpack(bnd, batch, s, s))
        assert np.max(e) <= 4 * 3 * max(s, 1) * U32, (ta, tb, s, np.max(e) / U32)
        h32, l32 = oracle.gemm_strided(ta, tb, s, s, s, 1.5, A, ra, ra * s, B, rb, rb * s, -0.5, C, s, s * s,
                                       batch, ext=True)
        b32 = oracle.bound_strided(ta, tb, s, s, s, 1.5, A, ra, ra * s, B, rb, rb * s, -0.5, C, s, s * s, batch)
        say(f"  end-to-end max normalised error vs fp32 inputs: {np.max(normalised_error(got, h32, l32, b32)):.3e}")


@pytest.mark.parametrize("mode", ["bf16", "f16", "e4m3", "bf16x3", "f32"])
def test_precision_modes_vbatched(gpu_lib, mode):
    """The variable-size workload shape in every precision mode: sizes as in
    the variable-size batch, pointer arrays, device binning."""
    g = inputs.rng(4, salt=14)
    dims = inputs.varsize_dims(g, 1500)
    c = VarCase(np.float32, "N", "N", dims, 1.5, -0.5, g, pad=False)
    d = c.device()
    N = c.batch
    kw = {}
    Ast, Bst = c.A, c.B
    if mode in ("bf16", "f16"):
        tdt, code = NARROW[mode]
        nA = d["A"].to(tdt)
        nB = d["B"].to(tdt)
        pA = torch.tensor(nA.data_ptr() + c.offA * 2, device="cuda")
        pB = torch.tensor(nB.data_ptr() + c.offB * 2, device="cuda")
        sA = sB = None
        cmode = sbg.MODE_PLAIN
        Ast = nA.view(torch.int16).cpu().numpy().view(np.uint16)
        Bst = nB.view(torch.int16).cpu().numpy().view(np.uint16)
        kw = dict(types=(mode, mode, "f32"))
    elif mode == "e4m3":
        code, cmode = sbg.R_8F_E4M3, sbg.MODE_PLAIN
        qA = torch.zeros(c.A.size, dtype=torch.uint8, device="cuda")
        qB = torch.zeros(c.B.size, dtype=torch.uint8, device="cuda")
        sA = torch.empty(N, dtype=torch.float32, device="cuda")
        sB = torch.empty(N, dtype=torch.float32, device="cuda")
        pA = torch.tensor(qA.data_ptr() + c.offA, device="cuda")
        pB = torch.tensor(qB.data_ptr() + c.offB, device="cuda")
        sbg.quantize_e4m3_vbatched(d["m"], d["k"], 16, 16, d["pA"], d["lda"], pA, d["lda"], sA, N)
        sbg.quantize_e4m3_vbatched(d["k"], d["n"], 16, 16, d["pB"], d["ldb"], pB, d["ldb"], sB, N)
        torch.cuda.synchronize()
        Ast, Bst = from_dev(qA), from_dev(qB)
        kw = dict(types=("e4m3", "e4m3", "f32"), scaleA=from_dev(sA).astype(np.float64),
                  scaleB=from_dev(sB).astype(np.float64))
    else:
        code = sbg.R_32F
        cmode = sbg.MODE_BF16X3 if mode == "bf16x3" else sbg.MODE_PLAIN
        pA, pB, sA, sB = d["pA"], d["pB"], None, None
    say(f"vbatched_ex {mode} N={N}")
    sbg.gemm_vbatched_ex("N", "N", d["m"], d["n"], d["k"], 16, 16, 16, 1.5, pA, d["lda"], sA, pB, d["ldb"], sB,
                         -0.5, d["pC"], d["ldc"], N, code, cmode, d["ws"])
    torch.cuda.synchronize()
    out = from_dev(d["C"])
    if mode == "bf16x3":
        hi, lo, bnd, offO, mm, nn = oracle.gemm_split3_general("N", "N", c.m, c.n, c.k, 1.5, c.A, c.offA, c.lda,
                                                               c.B, c.offB, c.ldb, -0.5, c.C, c.offC, c.ldc, N)
        for p in range(N):
            m, n = int(c.m[p]), int(c.n[p])
            if m == 0 or n == 0:
                continue
            o = int(offO[p])
            e = normalised_error(c.got(out, p), hi[o:o + m * n].reshape(n, m).T, lo[o:o + m * n].reshape(n, m).T,
                                 bnd[o:o + m * n].reshape(n, m).T)
            assert np.max(e) <= 12 * max(int(c.k[p]), 1) * U32, (p, np.max(e) / U32)
    else:
        check_var(c, out, label=f"vbatched_ex {mode}", A=Ast, B=Bst, **kw)


def test_ex_argument_checks(gpu_lib):
    """Precision arguments are validated after the GEMM arguments."""
    L = sbg.load()
    import ctypes
    one = (ctypes.c_float * 1)(1.0)
    a = ctypes.cast(one, ctypes.c_void_p)
    dev = torch.zeros(64, device="cuda")
    p = ctypes.c_void_p(dev.data_ptr())
    # fp8 without scales
    st = L.sbg_gemm_strided_batched_ex(b"N", b"N", 4, 4, 4, a, p, 4, 16, None, p, 4, 16, None, a, p, 4, 16, 1,
                                       sbg.R_8F_E4M3, sbg.MODE_PLAIN, None)
    assert st == sbg.SBG_INVALID_VALUE and sbg.last_invalid_arg() == 10
    # BF16x3 on bf16 storage
    st = L.sbg_gemm_strided_batched_ex(b"N", b"N", 4, 4, 4, a, p, 4, 16, None, p, 4, 16, None, a, p, 4, 16, 1,
                                       sbg.R_16BF, sbg.MODE_BF16X3, None)
    assert st == sbg.SBG_INVALID_VALUE and sbg.last_invalid_arg() == 21
    # unknown type
    st = L.sbg_gemm_strided_batched_ex(b"N", b"N", 4, 4, 4, a, p, 4, 16, None, p, 4, 16, None, a, p, 4, 16, 1,
                                       9, sbg.MODE_PLAIN, None)
    assert st == sbg.SBG_INVALID_VALUE and sbg.last_invalid_arg() == 20
    torch.cuda.synchronize()
