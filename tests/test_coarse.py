"""The coarse-level solver of the closed DNN-MG loop (paper_2008_11520_amd/
coarse.py), on the host:

* an exact steady Navier-Stokes solution that is affine in v and p (div v = 0,
  (v.grad)v + grad p = 0, Delta v = 0) lies in the Q1/Q1 spaces and is not
  touched by the stabilisation (grad p is constant), so with b = (1/dt) M v
  and its Dirichlet values Newton recovers it from zero, on perturbed meshes;
* the Newton Jacobian equals central differences of the residual;
* the stabilisation vanishes on affine pressures and not on the checkerboard;
* Poiseuille flow with a do-nothing outflow (an exact steady solution,
  quadratic in y, whose natural outflow condition holds) is reproduced at
  the nodes: the velocity by the nodal exactness of the 1D problem, the
  linear pressure exactly (the stabilisation does not act on it), which
  also pins the outflow's natural boundary treatment.
"""
import numpy as np
import pytest

from paper_2008_11520_amd import synth
from paper_2008_11520_amd.coarse import CoarseNS


def _affine(xy, a=0.3, b=0.7, d=-0.2):
    x, y = xy[:, 0], xy[:, 1]
    v = np.stack([a + b * (x + y), d - b * (x + y)], axis=1)
    p = -b * (a + d) * (x - y)
    return v, p


@pytest.mark.parametrize("nx,ny,seed", [(6, 5, 1), (9, 4, 2)])
def test_affine_exact_solution_is_recovered(nx, ny, seed):
    cxy = synth.perturb_interior(synth.rect_mesh(nx, ny, 2.2, 0.41), 0.1, seed)
    xy = cxy.reshape(-1, 2)
    ns = CoarseNS(cxy, 0.01, 1e-3, 15)
    v_ex, p_ex = _affine(xy)
    b = ns.mass_rhs(v_ex)
    v0 = np.where(ns.dmask[:, None], v_ex, 0.0)
    v, p, it = ns.solve(b, v_ex, v0, np.zeros(ns.N))
    assert it >= 2
    assert np.abs(v - v_ex).max() <= 1e-10 * np.abs(v_ex).max()
    assert np.abs(p - (p_ex - p_ex[0])).max() <= 1e-8 * np.abs(p_ex).max()


def test_newton_jacobian_matches_central_differences():
    nx, ny = 5, 4
    cxy = synth.perturb_interior(synth.rect_mesh(nx, ny, 2.2, 0.41), 0.1, 3)
    ns = CoarseNS(cxy, 0.01, 1e-2, synth.DIR_CHANNEL)
    rng = np.random.default_rng(4)
    v = rng.standard_normal((ns.N, 2))
    p = rng.standard_normal(ns.N)
    b = rng.standard_normal((ns.N, 2))
    vD = rng.standard_normal((ns.N, 2))
    d = rng.standard_normal(3 * ns.N)
    J = ns.jacobian(v)
    eps = 1e-6

    def F(x):
        return ns.residual(v + x[:2 * ns.N].reshape(2, ns.N).T, p + x[2 * ns.N:], b, vD)
    fd = (F(eps * d) - F(-eps * d)) / (2 * eps)
    assert np.abs(J @ d - fd).max() <= 1e-7 * np.abs(fd).max()


@pytest.mark.parametrize("nx,ny", [(6, 6), (7, 5)])
def test_stabilisation_vanishes_on_affine_pressure_only(nx, ny):
    """The stabilisation is symmetric positive semi-definite, zero on affine
    pressures (consistency) and positive on the checkerboard and on the
    column- and row-alternating modes (which a per-element mean gradient
    would not see)."""
    cxy = synth.perturb_interior(synth.rect_mesh(nx, ny), 0.1, 5)
    ns = CoarseNS(cxy, 0.01, 1e-3, 15)
    xy = cxy.reshape(-1, 2)
    S = ns.S.toarray()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() >= -1e-10 * np.abs(S).max()
    p_aff = 1.0 + 2.0 * xy[:, 0] - 3.0 * xy[:, 1]
    assert np.abs(S @ p_aff).max() <= 1e-12 * np.abs(S).max() * np.abs(p_aff).max()
    I = np.arange(ns.N) % (nx + 1)
    J = np.arange(ns.N) // (nx + 1)
    for mode in ((-1.0) ** (I + J), (-1.0) ** I, (-1.0) ** J):
        assert mode @ (S @ mode) > 1e-3 * np.abs(S).max()


def test_poiseuille_with_do_nothing_outflow_is_reproduced():
    U, H, L, nu = 1.0, 0.41, 2.2, 1e-2
    errs = []
    for n in (8, 16, 32):
        nx, ny = 2 * n, n
        cxy = synth.rect_mesh(nx, ny, L, H)
        xy = cxy.reshape(-1, 2)
        ns = CoarseNS(cxy, 1e8, nu, synth.DIR_CHANNEL)      # steady: dt -> infinity
        ux = U * 4 * xy[:, 1] * (H - xy[:, 1]) / H ** 2
        v_ex = np.stack([ux, 0 * ux], axis=1)
        p_ex = -8 * U * nu / H ** 2 * (xy[:, 0] - L)
        v, p, _ = ns.solve(np.zeros((ns.N, 2)), v_ex, np.where(ns.dmask[:, None], v_ex, 0.0), np.zeros(ns.N))
        errs.append((np.abs(v - v_ex).max(), np.abs(p - p_ex).max()))
    pmax = 8 * U * nu / H ** 2 * L
    assert max(e[0] for e in errs) < 1e-8 * U, errs
    assert max(e[1] for e in errs) < 1e-7 * pmax, errs


@pytest.mark.parametrize("nx,ny,seed", [(6, 5, 1), (9, 4, 2)])
def test_crank_nicolson_keeps_the_affine_steady_solution(nx, ny, seed):
    """Crank-Nicolson (theta = 1/2): from the steady solution u the right-hand
    side (1/dt) M u - (1/2) T(u) gives back v = u and the same pressure,
    since the discrete T(u) equals B^T p of the steady pressure."""
    cxy = synth.perturb_interior(synth.rect_mesh(nx, ny, 2.2, 0.41), 0.1, seed)
    xy = cxy.reshape(-1, 2)
    ns = CoarseNS(cxy, 0.2, 1e-3, 15, theta=0.5)     # dt large enough that T(u) shows beside M u / dt
    v_ex, p_ex = _affine(xy)
    b = ns.rhs_of(v_ex)
    assert np.abs(b - ns.mass_rhs(v_ex)).max() > 2e-3 * np.abs(b).max()   # the explicit term is there
    v0 = np.where(ns.dmask[:, None], v_ex, 0.0)
    v, p, it = ns.solve(b, v_ex, v0, np.zeros(ns.N))
    assert it >= 2
    assert np.abs(v - v_ex).max() <= 1e-10 * np.abs(v_ex).max()
    assert np.abs(p - (p_ex - p_ex[0])).max() <= 1e-8 * np.abs(p_ex).max()


def test_crank_nicolson_jacobian_matches_central_differences():
    nx, ny = 5, 4
    cxy = synth.perturb_interior(synth.rect_mesh(nx, ny, 2.2, 0.41), 0.1, 3)
    ns = CoarseNS(cxy, 0.01, 1e-2, synth.DIR_CHANNEL, theta=0.5)
    rng = np.random.default_rng(6)
    v = rng.standard_normal((ns.N, 2))
    p = rng.standard_normal(ns.N)
    b = rng.standard_normal((ns.N, 2))
    vD = rng.standard_normal((ns.N, 2))
    d = rng.standard_normal(3 * ns.N)
    eps = 1e-6

    def F(x):
        return ns.residual(v + x[:2 * ns.N].reshape(2, ns.N).T, p + x[2 * ns.N:], b, vD)
    fd = (F(eps * d) - F(-eps * d)) / (2 * eps)
    assert np.abs(ns.jacobian(v) @ d - fd).max() <= 1e-7 * np.abs(fd).max()


def test_theta_weights_the_transport_of_the_momentum_rows():
    """residual(theta) = M/dt v + theta T(v) - B^T p - b at free rows: the
    residual of theta = 1/2 is the mean of those of theta = 1 and theta = 0."""
    cxy = synth.perturb_interior(synth.rect_mesh(5, 4, 2.2, 0.41), 0.1, 8)
    rng = np.random.default_rng(9)
    ns = {t: CoarseNS(cxy, 0.01, 1e-2, synth.DIR_CHANNEL, theta=t) for t in (0.0, 0.5, 1.0)}
    N = ns[1.0].N
    v, p, b, vD = rng.standard_normal((N, 2)), rng.standard_normal(N), rng.standard_normal((N, 2)), rng.standard_normal((N, 2))
    r = {t: ns[t].residual(v, p, b, vD) for t in ns}
    assert np.abs(r[0.5] - 0.5 * (r[0.0] + r[1.0])).max() <= 1e-12 * np.abs(r[1.0]).max()
    assert np.abs(r[1.0] - r[0.0]).max() > 1e-3 * np.abs(r[1.0]).max()
