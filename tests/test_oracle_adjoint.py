"""Pins of the oracle's adjoint (VJP) of the P3M force and the leapfrog.

Everything here is checked against finite differences of the oracle's own
forward functions (the definition of a derivative, not a retyped formula),
and against invariants the exact transpose must satisfy: total momentum is
conserved by both force parts, so a uniform cotangent has a zero VJP; the
pair sum is translation invariant, so its VJP sums to zero.
"""
import numpy as np
import pytest

from oracle import adjoint, integrate
from oracle import pm as o_pm
from oracle import pp as o_pp
from oracle.split import split_factor

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _pp_case(n=24, seed=3):
    rng = np.random.default_rng(seed)
    pos = rng.random((3, n))
    m = rng.uniform(0.5, 1.5, n) / n
    return pos, m, 1.0, 0.06, 0.27, 0.01        # box, r_s, r_c = 4.5 r_s, eps


def _min_image(pos, box):
    d = pos[:, :, None] - pos[:, None, :]
    d -= box * np.round(d / box)
    return np.sqrt(np.einsum("dij,dij->ij", d, d))


def _fd_jacobian(fn, pos, delta):
    """Central-difference Jacobian dF/dx, shape (3N, 3N), of fn(pos) -> (3, N)."""
    n = pos.shape[1]
    J = np.zeros((3 * n, 3 * n))
    for k in range(n):
        for d in range(3):
            xp = pos.copy()
            xm = pos.copy()
            xp[d, k] += delta
            xm[d, k] -= delta
            J[:, d * n + k] = ((fn(xp) - fn(xm)) / (2 * delta)).reshape(-1)
    return J


def test_split_factor_derivative_matches_finite_differences():
    r_s = 0.7
    r = np.linspace(0.05, 6.0, 200) * r_s
    h = 1e-5 * r_s
    fd = (split_factor(r + h, r_s) - split_factor(r - h, r_s)) / (2 * h)
    np.testing.assert_allclose(adjoint.split_factor_derivative(r, r_s), fd, rtol=1e-7,
                               atol=1e-12)
    assert adjoint.split_factor_derivative(0.0, r_s) == 0.0     # f is flat at r = 0


def test_pp_vjp_is_the_transpose_of_the_finite_difference_jacobian():
    pos, m, box, r_s, r_c, eps = _pp_case()
    R = _min_image(pos, box)
    assert np.min(np.abs(R - r_c)) > 1e-4          # no pair within reach of the cutoff jump
    fn = lambda x: m * o_pp.pp_accel(x, m, box, r_s, r_c, eps, G=1.0, method="brute")
    J = _fd_jacobian(fn, pos, 1e-7)
    lam = np.random.default_rng(4).normal(size=pos.shape)
    ref = (J.T @ lam.reshape(-1)).reshape(3, -1)
    got = adjoint.pp_vjp(pos, m, box, r_s, r_c, eps, lam, G=1.0)
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_pp_vjp_invariants():
    pos, m, box, r_s, r_c, eps = _pp_case(n=200, seed=5)
    lam = np.random.default_rng(6).normal(size=pos.shape)
    got = adjoint.pp_vjp(pos, m, box, r_s, r_c, eps, lam, G=2.0)
    scale = np.max(np.abs(got))
    assert scale > 0
    assert np.max(np.abs(got.sum(axis=1))) <= 1e-12 * scale * pos.shape[1]    # translation
    uni = np.tile(np.array([[0.3], [-1.1], [0.7]]), (1, pos.shape[1]))
    assert np.max(np.abs(adjoint.pp_vjp(pos, m, box, r_s, r_c, eps, uni))) == 0.0
    # linear in lam and in G
    half = adjoint.pp_vjp(pos, m, box, r_s, r_c, eps, 0.5 * lam, G=1.0)
    np.testing.assert_allclose(half, 0.25 * got, rtol=1e-12, atol=1e-14 * scale)
    # the k-d tree pair set gives the same result as the all-pairs scan
    a = adjoint.pp_vjp(pos, m, box, r_s, r_c, eps, lam, method="brute")
    b = adjoint.pp_vjp(pos, m, box, r_s, r_c, eps, lam, method="kdtree")
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14 * scale)


def _pm_case(n=16, ng=8, seed=11):
    rng = np.random.default_rng(seed)
    h = 1.0 / ng
    # keep every coordinate at least 1e-3 h away from a node plane
    cells = rng.integers(0, ng, (3, n))
    frac = rng.uniform(0.01, 0.99, (3, n))
    pos = (cells + frac) * h
    m = rng.uniform(0.5, 1.5, n) / n
    return pos, m, 1.0, ng, 1.25 * h


@pytest.mark.parametrize("fd_order,deconv", [(4, 2), (2, 0)])
def test_pm_vjp_is_the_transpose_of_the_finite_difference_jacobian(fd_order, deconv):
    pos, m, box, ng, r_s = _pm_case()
    fn = lambda x: m * o_pm.pm_accel(x, m, box, ng, r_s, 1.0, fd_order, deconv)
    J = _fd_jacobian(fn, pos, 1e-7)
    lam = np.random.default_rng(12).normal(size=pos.shape)
    ref = (J.T @ lam.reshape(-1)).reshape(3, -1)
    got = adjoint.pm_vjp(pos, m, box, ng, r_s, lam, 1.0, fd_order, deconv)
    assert np.max(np.abs(got - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_pm_vjp_uniform_cotangent_is_zero():
    """sum_i F_i = 0 for the mesh force too (same CIC weights both ways, an
    antisymmetric difference and a symmetric Green's function), so
    d(sum_i c . F_i)/dx_k = 0."""
    pos, m, box, ng, r_s = _pm_case(n=300, ng=16, seed=13)
    lam = np.random.default_rng(14).normal(size=pos.shape)
    scale = np.max(np.abs(adjoint.pm_vjp(pos, m, box, ng, r_s, lam)))
    uni = np.tile(np.array([[1.3], [0.2], [-0.4]]), (1, pos.shape[1]))
    assert np.max(np.abs(adjoint.pm_vjp(pos, m, box, ng, r_s, uni))) <= 1e-12 * scale


def test_p3m_vjp_and_leapfrog_vjp_match_finite_differences():
    """The full force and a 3-step leapfrog: <mu, VJP(bar)> = <bar, JVP(mu)>
    with the JVP by central differences of the oracle's forward functions."""
    rng = np.random.default_rng(21)
    ng, n, box = 8, 20, 1.0
    h = box / ng
    pos = (rng.integers(0, ng, (3, n)) + rng.uniform(0.05, 0.95, (3, n))) * h
    mom = rng.normal(size=(3, n)) * 1e-3
    m = rng.uniform(0.5, 1.5, n) / n
    kw = dict(rs_cells=1.25, cutoff_rs=3.0, eps=0.02)        # r_c = 0.47 < L/2
    from oracle.p3m import p3m_accel

    def force(x):
        return m * p3m_accel(x, m, box, ng, kw["rs_cells"], kw["cutoff_rs"], kw["eps"],
                             pp_method="brute")

    lam = rng.normal(size=(3, n))
    mu = rng.normal(size=(3, n))
    d = 1e-7
    jvp = (force(pos + d * mu) - force(pos - d * mu)) / (2 * d)
    vjp = adjoint.p3m_vjp(pos, m, box, ng, lam, **kw)
    lhs, rhs = np.sum(mu * vjp), np.sum(lam * jvp)
    assert abs(lhs - rhs) <= 1e-6 * np.sum(np.abs(mu * vjp))

    dt, steps = 0.02, 3
    vjp_fn = lambda x, l: adjoint.p3m_vjp(x, m, box, ng, l, **kw)
    xs, pT = adjoint.leapfrog(pos, mom, m, force, dt, box, steps)
    xb, pb = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    x0b, p0b = adjoint.leapfrog_vjp(xs, m, vjp_fn, dt, xb, pb)
    mux, mup = rng.normal(size=(3, n)), rng.normal(size=(3, n))

    def run(e):
        ys, q = adjoint.leapfrog(pos + e * mux, mom + e * mup, m, force, dt, box, steps)
        return ys[-1], q

    (xp, pp_), (xm, pm_) = run(d), run(-d)
    rhs = np.sum(xb * (xp - xm) + pb * (pp_ - pm_)) / (2 * d)
    lhs = np.sum(x0b * mux + p0b * mup)
    assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + 1e-300)
    # the trajectory stayed inside the box faces (wrap has slope 1 elsewhere)
    assert all(np.all((x > 1e-6) & (x < box - 1e-6)) for x in xs)
    # a 1-step trajectory with F = 0 is a free drift: x_bar_0 = x_bar, p_bar_0 = p_bar + dt/m x_bar
    zero_vjp = lambda x, l: np.zeros_like(l)
    xs0 = [pos, integrate.drift(pos, mom, m, dt, box)]
    a, b = adjoint.leapfrog_vjp(xs0, m, zero_vjp, dt, xb, pb)
    np.testing.assert_array_equal(a, xb)
    np.testing.assert_allclose(b, pb + dt / m[None, :] * xb, rtol=1e-15)


def test_pp_vjp_on_targets_equals_the_full_columns():
    """The target-restricted short-range transpose (each target's own pairs
    from a k-d tree) gives the same columns as the all-pairs sum."""
    from paper_1510_07621_amd import ics
    rng = np.random.default_rng(6)
    pos = ics.uniform(3000, seed=5)
    m = rng.uniform(0.5, 1.5, 3000) / 3000
    lam = rng.normal(size=(3, 3000))
    r_s = 1.25 / 16
    full = adjoint.pp_vjp(pos, m, 1.0, r_s, 4.5 * r_s, 0.002, lam)
    tg = np.sort(rng.choice(3000, 200, replace=False))
    part = adjoint.pp_vjp(pos, m, 1.0, r_s, 4.5 * r_s, 0.002, lam, targets=tg)
    assert part.shape == (3, 200)
    assert np.max(np.abs(part - full[:, tg])) <= 1e-13 * np.max(np.abs(full))
