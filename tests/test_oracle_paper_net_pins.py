"""Pins of the oracle's paper-network form (inputs and head of Sec. 4.2,
architecture figure, parameter counts of Sec. 5.2 and 5.5) against values
the paper prints, closed forms and special cases.

Readings (the paper names the groups but not every detail): the continuity
rows are -(div Pv, xi_a) without the pressure stabilisation; the twelve
geometry values are edge lengths (bottom, right, top, left), aspect ratios
(h0/h1, h2/h3, h0/h2, h1/h3) and the interior angles at 00, 10, 11, 01; the
Peclet size q is the square root of the patch area; each convolutional block
is a 4-filter 3 x 3 convolution followed by its transpose with the same
weights (36 weights), the vertex block on the 2 x nf image of (component,
node), the spatial block on each component's (n+1) x (n+1) node grid; the
last layer sums the two blocks and weights every output entry.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2008_11520_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_parameter_counts_match_the_paper():
    g = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))
    one, two = g["one_level"], g["two_level"]
    # Sec. 5.2: 8634 at K = 1, N_GRU = 32 (GRU + FC + 2 x 36 + 18)
    assert oracle.paper_weight_count(one["K"], one["N_GRU"]) == one["total_params"]
    # Sec. 5.5: 60960 = GRU + FC at K = 2, N_GRU = 96; the count printed there
    # has no convolution weights, which this form adds (36 + 36 + 50)
    assert oracle.paper_weight_count(two["K"], two["N_GRU"]) == two["total_params"] + 36 + 36 + two["N_out"]
    for K, nin in ((1, one["N_in"]), (2, two["N_in"])):
        n = 1 << K
        assert 3 * (n + 1) ** 2 + 24 == nin


def _mesh(kind, nx=6, ny=4):
    if kind == "rect":
        return synth.rect_mesh(nx, ny, 2.2, 0.41)
    return synth.perturb_interior(synth.rect_mesh(nx, ny, 2.2, 0.41), 0.12, 7)


@pytest.mark.parametrize("kind", ["rect", "perturbed"])
@pytest.mark.parametrize("K", [1, 2])
def test_continuity_rows_vanish_for_divergence_free_affine_fields(kind, K):
    nx, ny = 6, 4
    cxy = _mesh(kind, nx, ny)
    xy = cxy.reshape(-1, 2)
    v = np.stack([0.3 + 1.7 * xy[:, 1] - 0.4 * xy[:, 0], -0.2 + 0.9 * xy[:, 0] + 0.4 * xy[:, 1]], axis=1)
    pv = oracle.prolong(nx, ny, K, v)
    Rp = oracle.continuity_rows(nx, ny, K, cxy.reshape(-1, 2), pv)
    assert np.abs(Rp).max() <= 1e-13 * np.abs(pv).max()


@pytest.mark.parametrize("kind", ["rect", "perturbed"])
@pytest.mark.parametrize("K", [1, 2])
def test_continuity_rows_of_a_constant_divergence_are_minus_the_mass_row_sums(kind, K):
    """v = (a x, b y): div v = a + b everywhere, so -(div v, xi_a) equals
    -(a + b) times the row sums of the consistent mass matrix."""
    nx, ny = 6, 4
    cxy = _mesh(kind, nx, ny)
    xy = cxy.reshape(-1, 2)
    a, b = 1.3, -0.4
    v = np.stack([a * xy[:, 0], b * xy[:, 1]], axis=1)
    pv = oracle.prolong(nx, ny, K, v)
    Rp = oracle.continuity_rows(nx, ny, K, cxy.reshape(-1, 2), pv)
    ones = np.ones_like(pv)
    M1 = oracle.mass_apply(nx, ny, K, cxy.reshape(-1, 2), ones)[:, 0]
    assert np.abs(Rp + (a + b) * M1).max() <= 1e-13 * np.abs(M1).max()


@pytest.mark.parametrize("K", [1, 2, 3])
def test_continuity_rows_sum_to_minus_the_exact_divergence_integral(K):
    """Rectangle [0, Lx] x [0, Ly]: coarse nodal values of a bilinear field
    v = (c0 + c1 x + c2 y + c3 x y, e0 + e1 x + e2 y + e3 x y) prolongate to
    the same field; the rows sum to -int div v = -(c1 Lx Ly + c3 Lx Ly^2 / 2
    + e2 Lx Ly + e3 Lx^2 Ly / 2)."""
    nx, ny, Lx, Ly = 5, 3, 2.2, 0.41
    cxy = synth.rect_mesh(nx, ny, Lx, Ly)
    x, y = cxy.reshape(-1, 2)[:, 0], cxy.reshape(-1, 2)[:, 1]
    c = (0.2, 1.1, -0.7, 2.3)
    e = (-0.5, 0.6, 0.9, -1.4)
    v = np.stack([c[0] + c[1] * x + c[2] * y + c[3] * x * y, e[0] + e[1] * x + e[2] * y + e[3] * x * y], axis=1)
    Rp = oracle.continuity_rows(nx, ny, K, cxy.reshape(-1, 2), oracle.prolong(nx, ny, K, v))
    exact = c[1] * Lx * Ly + c[3] * Lx * Ly ** 2 / 2 + e[2] * Lx * Ly + e[3] * Lx ** 2 * Ly / 2
    assert abs(Rp.sum() + exact) <= 1e-12 * abs(exact)


def test_geometry_of_known_cells():
    # a 2 x 1 grid: a square of side 0.5 and a parallelogram (0.5,0)-(2.5,0)-(3.5,1)-(1.5,1)
    # is not a grid; take one cell at a time
    sq = np.array([[[0.0, 0.0], [0.5, 0.0]], [[0.0, 0.5], [0.5, 0.5]]])
    G = oracle.paper_geometry(1, 1, sq.reshape(-1, 2))[0]
    assert np.allclose(G[:4], 0.5, rtol=0, atol=1e-15)
    assert np.allclose(G[4:8], 1.0, rtol=0, atol=1e-15)
    assert np.allclose(G[8:], math.pi / 2, rtol=0, atol=1e-15)
    # parallelogram: corners 00 (0,0), 10 (2,0), 11 (3,1), 01 (1,1)
    pg = np.array([[[0.0, 0.0], [2.0, 0.0]], [[1.0, 1.0], [3.0, 1.0]]])
    G = oracle.paper_geometry(1, 1, pg.reshape(-1, 2))[0]
    r2 = math.sqrt(2.0)
    assert np.allclose(G[:4], [2.0, r2, 2.0, r2], rtol=1e-15)
    assert np.allclose(G[4:8], [2.0 / r2, 2.0 / r2, 1.0, 1.0], rtol=1e-15)
    assert np.allclose(G[8:], [math.pi / 4, 3 * math.pi / 4, math.pi / 4, 3 * math.pi / 4], rtol=1e-15)
    # a trapezoid: 00 (0,0), 10 (4,0), 11 (3,1), 01 (0,1): right angles at 00, 01
    tz = np.array([[[0.0, 0.0], [4.0, 0.0]], [[0.0, 1.0], [3.0, 1.0]]])
    G = oracle.paper_geometry(1, 1, tz.reshape(-1, 2))[0]
    assert np.allclose(G[:4], [4.0, r2, 3.0, 1.0], rtol=1e-15)
    assert np.allclose(G[4:8], [4.0 / r2, 3.0, 4.0 / 3.0, r2], rtol=1e-15)
    assert np.allclose(G[8:], [math.pi / 2, math.pi / 4, 3 * math.pi / 4, math.pi / 2], rtol=1e-15)


def test_geometry_angles_sum_to_two_pi_on_perturbed_meshes():
    cxy = _mesh("perturbed", 7, 5)
    G = oracle.paper_geometry(7, 5, cxy.reshape(-1, 2))
    assert np.abs(G[:, 8:].sum(1) - 2 * math.pi).max() <= 1e-13
    # opposite-edge ratios are the products of the neighbouring ones with the
    # edge ratios around the cell: (h0/h1)(h1/h3) = h0/h3 and so on
    h = G[:, :4]
    assert np.allclose(G[:, 6], h[:, 0] / h[:, 2], rtol=1e-15)
    assert np.allclose(G[:, 4] * G[:, 7], h[:, 0] / h[:, 3], rtol=1e-14)


def test_peclet_closed_form():
    # 2 x 1 rectangle cells of 0.5 x 0.2: q = sqrt(0.1)
    cxy = synth.rect_mesh(2, 1, 1.0, 0.2)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((6, 2))
    nu = 2e-3
    Pe = oracle.peclet(2, 1, cxy.reshape(-1, 2), v, nu)
    q = math.sqrt(0.1)
    corners = [[0, 1, 3, 4], [1, 2, 4, 5]]
    for e in range(2):
        for k in range(4):
            assert abs(Pe[e, k] - q * math.hypot(*v[corners[e][k]]) / nu) <= 1e-13 * Pe[e, k]


def test_paper_input_layout():
    nx, ny, K = 3, 2, 1
    s = oracle.sizes(nx, ny, K)
    nf = s["nf"]
    D = np.arange(2 * s["Fn"], dtype=float).reshape(-1, 2) + 0.25
    Rp = -np.arange(s["Fn"], dtype=float) - 0.5
    v = 1000.0 + np.arange(2 * s["Nc"], dtype=float).reshape(-1, 2)
    Pe = 5000.0 + np.arange(4 * s["P"], dtype=float).reshape(-1, 4)
    G = 9000.0 + np.arange(12 * s["P"], dtype=float).reshape(-1, 12)
    X = oracle.gather_input_paper(nx, ny, K, D, Rp, v, Pe, G)
    assert X.shape == (s["P"], 51)
    n = 2
    for j in range(ny):
        for i in range(nx):
            e = j * nx + i
            for b in range(n + 1):
                for a in range(n + 1):
                    l, f = b * (n + 1) + a, (j * n + b) * (nx * n + 1) + i * n + a
                    assert X[e, 2 * l] == D[f, 0] and X[e, 2 * l + 1] == D[f, 1]
                    assert X[e, 2 * nf + l] == Rp[f]
            for k, (di, dj) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
                c = (j + dj) * (nx + 1) + i + di
                assert X[e, 3 * nf + 2 * k] == v[c, 0] and X[e, 3 * nf + 2 * k + 1] == v[c, 1]
                assert X[e, 3 * nf + 8 + k] == Pe[e, k]
            assert np.array_equal(X[e, 3 * nf + 12:], G[e])


def _gru_weights(rng, nin, H):
    return [rng.standard_normal((H, nin)) * 0.5 for _ in range(3)] + [rng.standard_normal((H, H)) * 0.5 for _ in range(3)]


def test_gru_reset_after_special_cases():
    rng = np.random.default_rng(5)
    P, nin, H = 7, 5, 4
    X = rng.standard_normal((P, nin))
    h = rng.standard_normal((P, H))
    W = _gru_weights(rng, nin, H)
    # a diagonal U_h: r_k (U_h h)_k = U_h,kk r_k h_k, the two forms agree
    Wd = W[:5] + [np.diag(rng.standard_normal(H))]
    assert np.allclose(oracle.gru_form(X, h, *Wd, False), oracle.gru_form(X, h, *Wd, True), rtol=0, atol=1e-15)
    # h = 0: no U term at all, both forms agree
    z0 = np.zeros((P, H))
    assert np.allclose(oracle.gru_form(X, z0, *W, False), oracle.gru_form(X, z0, *W, True), rtol=0, atol=1e-15)
    # in general they differ
    assert np.abs(oracle.gru_form(X, h, *W, False) - oracle.gru_form(X, h, *W, True)).max() > 1e-3
    # two units, state (0, 1), U_h = [[0, u], [0, 0]]: unit 0's candidate is
    # tanh(W_h x + u r_1) as printed and tanh(W_h x + r_0 u) with the reset after
    Wz, Wr, Wh = (rng.standard_normal((2, 3)) for _ in range(3))
    Uz, Ur = rng.standard_normal((2, 2)), rng.standard_normal((2, 2))
    u = 1.7
    Uh = np.array([[0.0, u], [0.0, 0.0]])
    x = rng.standard_normal((1, 3))
    hs = np.array([[0.0, 1.0]])
    sig = lambda t: 1.0 / (1.0 + math.exp(-t))
    z0_ = sig(Wz[0] @ x[0] + Uz[0] @ hs[0])
    r = [sig(Wr[k] @ x[0] + Ur[k] @ hs[0]) for k in range(2)]
    printed = (1 - z0_) * math.tanh(Wh[0] @ x[0] + u * r[1])
    after = (1 - z0_) * math.tanh(Wh[0] @ x[0] + r[0] * u)
    assert abs(oracle.gru_form(x, hs, Wz, Wr, Wh, Uz, Ur, Uh, False)[0, 0] - printed) <= 1e-15
    assert abs(oracle.gru_form(x, hs, Wz, Wr, Wh, Uz, Ur, Uh, True)[0, 0] - after) <= 1e-15


def _delta(dr=0, dc=0, f=0, scale=1.0):
    W = np.zeros(36)
    W[9 * f + 3 * (dr + 1) + (dc + 1)] = scale
    return W


@pytest.mark.parametrize("K", [1, 2])
def test_conv_head_identity_and_output_weights(K):
    """A centre-tap kernel makes a block the identity (conv and transposed
    conv of a delta); the head is then wf * (M h) per block used."""
    rng = np.random.default_rng(8)
    n = 1 << K
    nout, H, P = 2 * (n + 1) ** 2, 6, 5
    M = rng.standard_normal((nout, H))
    h = rng.standard_normal((P, H))
    wf = rng.standard_normal(nout)
    y = h @ M.T
    zero = np.zeros(36)
    for WV, WS, k in ((_delta(), zero, 1.0), (zero, _delta(f=2), 1.0), (_delta(f=3), _delta(f=1), 2.0)):
        d = oracle.conv_head(K, h, M, WV, WS, wf)
        assert np.allclose(d, k * y * wf, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("K", [1, 2])
def test_conv_head_shift_taps_zero_one_edge(K):
    """One off-centre tap: the convolution shifts, its transpose shifts back,
    so the block keeps its input except on the edge the shift pushes out.
    Spatial block, tap one column to the right: the node column a = 0 of each
    component becomes zero.  Vertex block, tap one row down (component
    axis): component 0 becomes zero."""
    rng = np.random.default_rng(9)
    n = 1 << K
    nf = (n + 1) ** 2
    nout, P = 2 * nf, 4
    M = np.eye(nout)
    h = rng.standard_normal((P, nout))
    ones, zero = np.ones(nout), np.zeros(36)
    d = oracle.conv_head(K, h, M, zero, _delta(dc=1), ones)
    keep = np.array([(l % (n + 1)) != 0 for l in range(nf) for c in range(2)])
    assert np.array_equal(d[:, ~keep], np.zeros_like(d[:, ~keep]))
    assert np.allclose(d[:, keep], h[:, keep], rtol=0, atol=1e-15)
    d = oracle.conv_head(K, h, M, _delta(dr=1), zero, ones)
    comp = np.array([c for l in range(nf) for c in range(2)])
    assert np.array_equal(d[:, comp == 0], np.zeros_like(d[:, comp == 0]))
    assert np.allclose(d[:, comp == 1], h[:, comp == 1], rtol=0, atol=1e-15)


def test_conv_blocks_are_symmetric_positive_semidefinite():
    """The second layer is the first one's transpose, so each block is
    W^T W: symmetric and positive semi-definite."""
    K = 1
    nout = 18
    rng = np.random.default_rng(10)
    WV, WS = rng.standard_normal(36), rng.standard_normal(36)
    E = np.eye(nout)
    for wv, ws in ((WV, np.zeros(36)), (np.zeros(36), WS)):
        B = oracle.conv_head(K, E, E, wv, ws, np.ones(nout)).T     # column i = block(e_i)
        assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
        assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() >= -1e-12 * np.abs(B).max()


def test_paper_step_wiring_and_zero_weights():
    """One paper-form step: its network input and correction are the
    compositions of the pinned pieces; with zero weights the correction is
    zero and b_L is that of the plain prolongation."""
    flow = synth.channel_flow(7, 4, 3, 0.005, perturb_seed=2)
    K, H, nu = 1, 8, 1e-3
    n = 2
    nf, nin, nout = 9, 51, 18
    rng = np.random.default_rng(12)
    w = rng.standard_normal(oracle.paper_weight_count(K, H)) * 0.3
    o = oracle.OracleFlow(flow.nx, flow.ny, K, H, 0, flow.dt, nu, flow.dirichlet, flow.cxy, w, form=1,
                          reset_after=True)
    v, p = flow.fields(0)
    o.step(v, p)
    v, p = flow.fields(1)
    h0 = o.h.copy()
    out = o.step(v, p, want=("Pv", "D", "X", "dpatch"))
    cxy = flow.cxy.reshape(-1, 2)
    Rp = oracle.continuity_rows(flow.nx, flow.ny, K, cxy, out["Pv"])
    X = oracle.gather_input_paper(flow.nx, flow.ny, K, out["D"], Rp, v, oracle.peclet(flow.nx, flow.ny, cxy, v, nu),
                                  oracle.paper_geometry(flow.nx, flow.ny, cxy))
    assert np.array_equal(out["X"], X)
    ws = np.split(w, np.cumsum([H * nin] * 3 + [H * H] * 3 + [nout * H, 36, 36]))
    Wz, Wr, Wh = (a.reshape(H, nin) for a in ws[:3])
    Uz, Ur, Uh = (a.reshape(H, H) for a in ws[3:6])
    hn = oracle.gru_form(X, h0, Wz, Wr, Wh, Uz, Ur, Uh, True)
    assert np.array_equal(o.h, hn)
    d = oracle.conv_head(K, hn, ws[6].reshape(nout, H), ws[7], ws[8], ws[9])
    assert np.array_equal(out["dpatch"], d)
    o0 = oracle.OracleFlow(flow.nx, flow.ny, K, H, 0, flow.dt, nu, flow.dirichlet, flow.cxy, np.zeros_like(w), form=1)
    r = o0.step(v, p, want=("Dbar", "bL"))
    assert np.all(r["Dbar"] == 0.0)
    b = oracle.rhs_restrict(flow.nx, flow.ny, K, cxy, v, np.zeros((oracle.sizes(flow.nx, flow.ny, K)["Fn"], 2)), flow.dt)
    assert np.array_equal(r["bL"], b)
    assert n == 1 << K and nf == (n + 1) ** 2
