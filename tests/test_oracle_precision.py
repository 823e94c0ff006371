"""Pins of the oracle's precision-mode parts (no GPU): the narrow-format
decoders, the E4M3 encoder and per-matrix quantiser, the bfloat16 rounding and
the BF16x3 reference, each tied to a library conversion or an exact special
case."""
import numpy as np
import pytest
import torch

import oracle
from paper_1304_7053_amd import inputs


def test_e4m3_decoder_matches_torch_for_all_codes():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    mine = np.array([oracle.decode(c, "e4m3") for c in range(256)])
    assert np.array_equal(np.isnan(ref), np.isnan(mine))
    ok = ~np.isnan(ref)
    assert np.array_equal(ref[ok], mine[ok])
    assert mine[0x7E] == 448.0 and mine[0x01] == 2.0 ** -9


def test_f16_and_bf16_decoders_match_library():
    h = np.arange(65536, dtype=np.uint16)
    ref16 = h.view(np.float16).astype(np.float64)
    mine16 = np.array([oracle.decode(c, "f16") for c in range(0, 65536, 7)])
    r = ref16[::7]
    assert np.array_equal(np.isnan(r), np.isnan(mine16))
    assert np.array_equal(r[~np.isnan(r)], mine16[~np.isnan(r)])
    refbf = torch.from_numpy(h.astype(np.int32)).to(torch.int16).view(torch.bfloat16).float().numpy()
    minebf = np.array([oracle.decode(c, "bf16") for c in range(0, 65536, 7)])
    rb = refbf[::7].astype(np.float64)
    assert np.array_equal(rb[~np.isnan(rb)], minebf[~np.isnan(rb)])


def test_e4m3_encoder_matches_torch_round_to_nearest_even():
    g = inputs.rng(301)
    x = np.concatenate([
        g.uniform(-448, 448, 20000),
        g.uniform(-2.0 ** -5, 2.0 ** -5, 20000),      # subnormal region
        # exact ties between neighbouring codes (midpoints) in several binades
        np.array([(a + b) / 2 for a, b in zip(
            [oracle.decode(c, "e4m3") for c in range(0, 0x7E)],
            [oracle.decode(c, "e4m3") for c in range(1, 0x7F)])]),
    ]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    mine = np.array([oracle.encode_e4m3(v) for v in x], dtype=np.uint8)
    assert np.array_equal(ref, mine)


def test_e4m3_encoder_saturates_finite_values():
    assert oracle.encode_e4m3(460.0) == 0x7E          # rounds down to 448
    assert oracle.encode_e4m3(464.0) == 0x7E          # tie: even code 448
    assert oracle.encode_e4m3(1e6) == 0x7E            # saturating, not NaN
    assert oracle.encode_e4m3(-1e6) == 0xFE
    assert oracle.encode_e4m3(float("nan")) & 0x7F == 0x7F


def test_bf16_rounding_matches_torch():
    g = inputs.rng(302)
    x = (g.standard_normal(50000) * 10.0 ** g.uniform(-30, 30, 50000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    mine = np.array([oracle.round_bf16(v) for v in x])
    assert np.array_equal(ref, mine)
    # tiny values: bfloat16 subnormals (spacing 2^-133)
    t = np.float32([2.0 ** -130 * 1.3, -(2.0 ** -128) * 1.7, 2.0 ** -133 * 0.5, 2.0 ** -133 * 1.5])
    assert np.array_equal(torch.from_numpy(t).to(torch.bfloat16).float().numpy().astype(np.float64),
                          np.array([oracle.round_bf16(v) for v in t]))


def test_quantiser_scale_and_codes():
    g = inputs.rng(303)
    batch, rows, cols, ld = 50, 7, 5, 9
    X = inputs.strided_batch(g, batch, rows, cols, ld, ld * cols + 2, np.float32, fill=1e30)
    X[: ld * cols + 2] = np.where(np.isfinite(X[: ld * cols + 2]) & (X[: ld * cols + 2] < 1e29), 0.0,
                                  X[: ld * cols + 2])            # matrix 0 all zero -> scale 1
    off = np.arange(batch, dtype=np.int64) * (ld * cols + 2)
    Q, offQ, scales = oracle.quant_e4m3(X, off, rows, cols, ld, batch)
    for p in range(batch):
        M = np.array([[X[off[p] + i + ld * j] for j in range(cols)] for i in range(rows)], dtype=np.float32)
        amax = np.float32(np.max(np.abs(M)))
        s = np.float32(1.0) if amax == 0 else np.float32(amax / np.float32(448.0))
        assert scales[p] == s
        ref = torch.from_numpy((M / s).astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
        got = Q[offQ[p]: offQ[p] + rows * cols].reshape(cols, rows).T
        assert np.array_equal(got, ref)
        if amax > 0:
            # the largest entry maps to +-448 exactly
            assert 0x7E in (got & 0x7F)


def test_split3_reduces_to_plain_gemm_on_bf16_values():
    """Inputs that are exact bfloat16 values have lo = 0, so the BF16x3 product
    is the plain product of the same numbers."""
    g = inputs.rng(304)
    m, n, k, batch = 6, 5, 9, 4
    A = torch.from_numpy(g.uniform(-1, 1, (batch, m, k)).astype(np.float32)).to(torch.bfloat16).float().numpy()
    B = torch.from_numpy(g.uniform(-1, 1, (batch, k, n)).astype(np.float32)).to(torch.bfloat16).float().numpy()
    C = g.uniform(-1, 1, (batch, m, n)).astype(np.float32)
    Af = np.swapaxes(A, 1, 2).reshape(-1)
    Bf = np.swapaxes(B, 1, 2).reshape(-1)
    Cf = np.swapaxes(C, 1, 2).reshape(-1)
    p = np.arange(batch)
    hi, lo, bnd, offO, _, _ = oracle.gemm_split3_general("N", "N", m, n, k, 1.5, Af, p * m * k, m, Bf, p * k * n, k,
                                                         -0.5, Cf, p * m * n, m, batch)
    rh, rl = oracle.gemm("N", "N", 1.5, A, B, -0.5, C, ext=True)
    got = np.swapaxes((hi + lo).reshape(batch, n, m), 1, 2)
    assert np.allclose(got, rh + rl, rtol=0, atol=1e-15)


def test_split3_recovers_fp32_products_to_bf16x3_accuracy():
    """x = hi + lo + r with |r| <= 2^-17 |x| (two 8-bit roundings); the dropped
    lo*lo and r terms bound the error of the split product against the exact
    product by about 2^-15 * sum |a||b|."""
    g = inputs.rng(305)
    m, n, k, batch = 16, 16, 16, 3
    A = g.uniform(-1, 1, (batch, m, k)).astype(np.float32)
    B = g.uniform(-1, 1, (batch, k, n)).astype(np.float32)
    C = np.zeros((batch, m, n), dtype=np.float32)
    p = np.arange(batch)
    hi, lo, bnd, _, _, _ = oracle.gemm_split3_general(
        "T", "T", m, n, k, 1.0, np.swapaxes(np.swapaxes(A, 1, 2), 1, 2).reshape(-1), p * m * k, k,
        np.swapaxes(np.swapaxes(B, 1, 2), 1, 2).reshape(-1), p * k * n, n, 0.0, C.reshape(-1), p * m * n, m, batch)
    # op T on row-major-flattened (batch, rows, cols) storage = op N on the matrices
    exact = np.einsum("bik,bkj->bij", A.astype(np.float64), B.astype(np.float64))
    absprod = np.einsum("bik,bkj->bij", np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64)))
    got = np.swapaxes((hi + lo).reshape(batch, n, m), 1, 2)
    err = np.abs(got - exact) / absprod
    assert np.max(err) < 2.0 ** -15
    assert np.max(err) > 2.0 ** -30   # the split is not exact for general binary32 data
