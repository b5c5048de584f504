"""Pins of the oracle's FP8 E4M3 operand form, each against something fixed
outside the oracle: the OCP E4M3 format's published extreme values and its
structure (8 equally spaced values per binade, monotone codes), brute-force
nearest-value search over all 256 codes, the quantiser's error bound, and
reductions to the FP64 network on operands that quantise exactly.

Beyond these the numerical values of the FP8 network for general operands
are "parity unpinned": only GPU <-> oracle agreement covers them."""
import math

import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import synth

FINITE = [c for c in range(256) if (c & 0x7F) != 0x7F]


def test_e4m3_published_values():
    # OCP 8-bit FP spec, E4M3: max normal 448 = S.1111.110, min normal 2^-6,
    # max subnormal 0.875 * 2^-6, min subnormal 2^-9, NaN S.1111.111, no inf
    assert oracle.e4m3_decode(0x7E) == 448.0
    assert oracle.e4m3_decode(0xFE) == -448.0
    assert oracle.e4m3_decode(0x08) == 2.0 ** -6
    assert oracle.e4m3_decode(0x07) == 0.875 * 2.0 ** -6
    assert oracle.e4m3_decode(0x01) == 2.0 ** -9
    assert oracle.e4m3_decode(0x38) == 1.0
    assert oracle.e4m3_decode(0x00) == 0.0 and math.copysign(1.0, oracle.e4m3_decode(0x80)) == -1.0
    assert math.isnan(oracle.e4m3_decode(0x7F)) and math.isnan(oracle.e4m3_decode(0xFF))


def test_e4m3_structure():
    pos = [oracle.e4m3_decode(c) for c in range(0x7F)]
    assert all(b > a for a, b in zip(pos, pos[1:]))               # monotone in the code
    for c in range(0x80):
        if c != 0x7F:
            assert oracle.e4m3_decode(c | 0x80) == -oracle.e4m3_decode(c)
    # each binade [2^e, 2^(e+1)) holds exactly 8 equally spaced values
    for e in range(-6, 9):
        vals = [v for v in pos if 2.0 ** e <= v < 2.0 ** (e + 1)]
        assert len(vals) == (7 if e == 8 else 8)
        steps = np.diff(vals)
        assert np.all(steps == 2.0 ** (e - 3))
    # subnormals: 2^-9 steps below the smallest normal
    sub = [v for v in pos if v < 2.0 ** -6]
    assert np.array_equal(np.diff(sub), np.full(len(sub) - 1, 2.0 ** -9))


def test_encode_fixed_points_and_ties_to_even():
    for c in FINITE:
        v = oracle.e4m3_decode(c)
        assert oracle.e4m3_encode(np.float32(v)) == c, hex(c)
    pos = [(c, oracle.e4m3_decode(c)) for c in range(0x7F)]
    for (c0, v0), (c1, v1) in zip(pos, pos[1:]):
        mid = np.float32((v0 + v1) / 2)
        assert float(mid) == (v0 + v1) / 2                           # midpoints are exact in FP32
        even = c0 if c0 % 2 == 0 else c1
        assert oracle.e4m3_encode(mid) == even, (hex(c0), hex(c1))
        assert oracle.e4m3_encode(np.nextafter(mid, np.float32(0))) == c0
        assert oracle.e4m3_encode(np.nextafter(mid, np.float32(1e9))) == c1


def test_encode_is_brute_force_nearest_and_saturates():
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.uniform(-4, 2.5, 3000),
                         rng.uniform(-500, 500, 500)]).astype(np.float32)
    table = np.array([oracle.e4m3_decode(c) for c in FINITE])
    codes = np.array(FINITE)
    for x in xs:
        if abs(x) >= 448:
            assert oracle.e4m3_encode(x) == (0xFE if x < 0 else 0x7E)
            continue
        d = np.abs(table - float(x))
        best = codes[d == d.min()]
        got = oracle.e4m3_encode(x)
        if x == 0:
            continue
        assert got in best or (len(best) > 1), (x, got, best)
        assert abs(oracle.e4m3_decode(got) - float(x)) == d.min()
    for big in (448.5, 463.9, 464.0, 1e6, np.inf):
        assert oracle.e4m3_encode(np.float32(big)) == 0x7E
        assert oracle.e4m3_encode(np.float32(-big)) == 0xFE


def test_quantiser_bound_and_scale():
    rng = np.random.default_rng(3)
    a = (rng.standard_normal((64, 104)) * np.exp(rng.uniform(-6, 6, (64, 1)))).astype(np.float32)
    a[5] = 0.0                                                       # an all-zero row
    q, s = oracle.quantize_rows(a)
    deq = np.vectorize(oracle.e4m3_decode)(q) * s[:, None].astype(np.float64)
    m = np.abs(a).max(axis=1).astype(np.float64)
    for i in range(a.shape[0]):
        if m[i] == 0:
            assert np.all(q[i] == 0) and s[i] > 0
            continue
        assert s[i] == np.float32(np.float32(m[i]) / np.float32(448.0))
        # the largest element maps to +-448
        j = int(np.argmax(np.abs(a[i])))
        assert q[i, j] & 0x7F == 0x7E
        ai = a[i].astype(np.float64)
        normal = np.abs(ai) / s[i] >= 2.0 ** -6
        # relative bound 2^-4 (half an ulp of a 3-bit mantissa), plus the FP32
        # rounding of a * r and of s
        err = np.abs(ai - deq[i])
        assert np.all(err[normal] <= (2.0 ** -4 + 1e-6) * np.abs(ai[normal]))
        assert np.all(err[~normal] <= (2.0 ** -10 + 1e-9) * s[i])


def _on_grid(rng, rows, cols, k, positive=False, lo=0x20):
    """Rows of E4M3 values times 2^k whose largest magnitude is 448 * 2^k."""
    codes = rng.integers(lo, 0x7E, size=(rows, cols))
    v = np.vectorize(oracle.e4m3_decode)(codes) * 2.0 ** k
    if not positive:
        v *= rng.choice([-1.0, 1.0], size=v.shape)
    j = rng.integers(0, cols, size=rows)
    v[np.arange(rows), j] = 448.0 * 2.0 ** k
    return v


def test_qgemm_exact_on_grid_and_error_bound():
    rng = np.random.default_rng(11)
    A, B = _on_grid(rng, 8, 40, -9), _on_grid(rng, 6, 40, -3)
    np.testing.assert_allclose(oracle.qgemm(A, B), A @ B.T, rtol=1e-15, atol=0)
    A = rng.standard_normal((16, 96)).astype(np.float32).astype(np.float64)
    B = rng.standard_normal((12, 96)).astype(np.float32).astype(np.float64)
    Q = oracle.qgemm(A, B)
    bound = np.abs(A) @ np.abs(B).T * ((1 + 2.0 ** -4) ** 2 - 1 + 1e-6) + 96 * 2.0 ** -10 * \
        (np.abs(A).max(1)[:, None] / 448) * np.abs(B).max() * 2
    assert np.all(np.abs(Q - A @ B.T) <= bound)
    assert np.abs(Q - A @ B.T).max() > 0                         # really quantised


def test_gru_fp8_reduces_to_fp64_on_exact_operands():
    """Operands on the E4M3 grid with row maxima 448 * 2^k quantise exactly;
    a reset gate driven to 1.0 (positive inputs and weights) makes r*h = h
    exact as well, so the FP8 GRU equals the FP64 one up to summation order."""
    rng = np.random.default_rng(5)
    P, nin, H = 6, 40, 32
    X = _on_grid(rng, P, nin, -2, positive=True, lo=0x50)          # every x >= 2
    h = _on_grid(rng, P, H, -9)
    Wz = _on_grid(rng, H, nin + H, -14)
    Wr = np.concatenate([_on_grid(rng, H, nin, -2, positive=True, lo=0x50), np.zeros((H, H))], axis=1)
    Wh = _on_grid(rng, H, nin, -14)
    Uh = _on_grid(rng, H, H, -5)
    args = (X, h, Wz[:, :nin], Wr[:, :nin], Wh, Wz[:, nin:], Wr[:, nin:], Uh)
    # the reset gate really saturates
    ar = X @ Wr[:, :nin].T + h @ Wr[:, nin:].T
    assert ar.min() > 40.0
    np.testing.assert_allclose(oracle.gru_fp8(*args), oracle.gru(*args), rtol=1e-13, atol=1e-15)
    # and a mistake-sensitive control: general operands do differ
    args2 = (X * (1.0 + 0.05 * rng.random(X.shape)), h) + args[2:]
    assert np.abs(oracle.gru_fp8(*args2) - oracle.gru(*args2)).max() > 1e-6


def test_mlp_fp8_reduces_to_fp64_on_exact_operands():
    rng = np.random.default_rng(9)
    P, H, nout = 5, 32, 18
    # h: powers of two plus one element 448 * 2^-8 that fixes the row scale
    e = rng.integers(-7, 0, size=(P, H))
    h = rng.choice([-1.0, 1.0], size=(P, H)) * 2.0 ** e
    h[:, 0] = 448.0 * 2.0 ** -8
    # M1: each row one weight 448 * 2^-3 on a column >= 1, so M1 h is 448 * 2^(e-3)
    Hm = H
    M1 = np.zeros((Hm, H))
    cols = rng.integers(1, H, size=Hm)
    M1[np.arange(Hm), cols] = 448.0 * 2.0 ** -3
    a = np.maximum(h @ M1.T, 0.0)
    assert np.all(a.max(axis=1) > 0)
    M2 = _on_grid(rng, nout, Hm, -6)
    np.testing.assert_allclose(oracle.mlp_fp8(h, M1, M2), oracle.mlp(h, M1, M2), rtol=1e-13, atol=1e-15)
    M = _on_grid(rng, nout, H, -2)
    np.testing.assert_allclose(oracle.mlp_fp8(h, M), oracle.mlp(h, M), rtol=1e-13, atol=1e-15)


def test_fp8_step_close_to_fp64_step():
    """The FP8 form is a perturbation of the FP64 step of the size the
    quantiser bound allows (a few per cent), and it is really applied."""
    flow = synth.channel_flow(6, 3, 2, 0.005, perturb_seed=4)
    K, H, Hm = 2, 64, 64
    w = synth.xavier_weights(K, H, Hm, 1234).astype(np.float64)
    o64 = oracle.OracleFlow(flow.nx, flow.ny, K, H, Hm, flow.dt, 1e-3, flow.dirichlet, flow.cxy, w)
    o8 = oracle.OracleFlow(flow.nx, flow.ny, K, H, Hm, flow.dt, 1e-3, flow.dirichlet, flow.cxy, w, fp8=True)
    for n in range(3):
        v, p = flow.fields(n)
        a = o64.step(v, p, want=("Dbar", "bL"))
        b = o8.step(v, p, want=("Dbar", "bL"))
        rel = np.linalg.norm(b["Dbar"] - a["Dbar"]) / np.linalg.norm(a["Dbar"])
        assert 1e-4 < rel < 0.15, rel
