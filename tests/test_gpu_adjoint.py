"""GPU parity of the force adjoint and the differentiable leapfrog.

The HIP path through the C ABI (p3m_force_vjp, pm_force_vjp, pp_force_vjp,
p3m_drift_vjp) against the oracle's transposes (oracle.adjoint), which are
pinned by finite differences on the CPU. Tolerances (per-particle relative
error of pos_bar, RMS): FP64 1e-9, FP32 1e-4; the drift transpose bit for
bit. Also: the GPU's own finite differences (<mu, VJP(lam)> = <lam, JVP(mu)>
with FP64 forces), conservation invariants, and torch.autograd through
autodiff.force and autodiff.leapfrog (with and without checkpointing).
"""
import numpy as np
import pytest
import torch

from oracle import adjoint, metrics
from paper_1510_07621_amd import ics

from _gpu import dev, host, plan, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _err(got, ref):
    return metrics.force_errors(got, ref)["rms"]


GRID = 16
H = 1.0 / GRID
EPS = 0.03 * H
KW = dict(rs_cells=1.25, cutoff_rs=4.5, eps=EPS, G=1.0)


@pytest.fixture(scope="module")
def case():
    """4096 particles on a 16^3 grid (one per cell on average) plus 200 close
    companions; per-particle masses; a random cotangent."""
    rng = np.random.default_rng(41)
    base = ics.uniform(4096, seed=42)
    near = (base[:, :200] + rng.uniform(0.05, 0.3, (3, 200)) * H) % 1.0
    pos = np.concatenate([base, near], axis=1)
    n = pos.shape[1]
    m = rng.uniform(0.5, 1.5, n) / n
    lam = rng.normal(size=(3, n))
    r_s = 1.25 * H
    r_c = 4.5 * r_s
    pp = adjoint.pp_vjp(pos, m, 1.0, r_s, r_c, EPS, lam)
    pm = adjoint.pm_vjp(pos, m, 1.0, GRID, r_s, lam)
    return pos, m, lam, pp, pm


def _vjp_plan(n, precision, **kw):
    return plan(GRID, n, precision, softening=EPS, adjoint=True, **kw)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_force_vjp_parity(case, precision, tol):
    pos, m, lam, pp, pm = case
    with _vjp_plan(pos.shape[1], precision) as P:
        x, mm, l = dev(pos), dev(m), dev(lam)
        got_pp = host(P.pp_force_vjp(x, mm, l))
        got_pm = host(P.pm_force_vjp(x, mm, l))
        got = host(P.force_vjp(x, mm, l))
    assert _err(got_pp, pp) <= tol
    assert _err(got_pm, pm) <= tol
    assert _err(got, pp + pm) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_force_vjp_one_sided_on_dense_groups(precision, tol):
    """The adjoint's pair sum evaluated once per pair between dense groups
    (pair_partials 80: the cotangent reactions gathered from partials)
    against the oracle's transpose, on dense cells of 400 and 600 particles
    in neighbouring groups plus a uniform background, per-particle masses;
    the scalar-mass path and the full adjoint with the mesh part too."""
    rng = np.random.default_rng(83)
    dense = np.concatenate([(np.array([3, 5, 7])[:, None] + rng.random((3, 400))) * H,
                            (np.array([4, 5, 8])[:, None] + rng.random((3, 600))) * H], axis=1)
    pos = np.concatenate([dense, ics.uniform(1200, seed=84)], axis=1)
    n = pos.shape[1]
    m = rng.uniform(0.5, 1.5, n) / n
    lam = rng.normal(size=(3, n))
    eps = 0.03 * H
    r_s = 1.25 * H
    ref = adjoint.pp_vjp(pos, m, 1.0, r_s, 4.5 * r_s, eps, lam)
    ref_s = adjoint.pp_vjp(pos, 1.0 / n, 1.0, r_s, 4.5 * r_s, eps, lam)
    ref_pm = adjoint.pm_vjp(pos, m, 1.0, GRID, r_s, lam)
    with plan(GRID, n, precision, softening=eps, adjoint=True, pair_partials=80) as P:
        got = host(P.pp_force_vjp(dev(pos), dev(m), dev(lam)))
        got_s = host(P.pp_force_vjp(dev(pos), 1.0 / n, dev(lam)))
        full = host(P.force_vjp(dev(pos), dev(m), dev(lam)))
    assert _err(got, ref) <= tol
    assert _err(got_s, ref_s) <= tol
    assert _err(full, ref + ref_pm) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
@pytest.mark.parametrize("soft_cells", [0.0, 0.03])
def test_coincident_particles_contribute_nothing(precision, tol, soft_cells):
    """Exact duplicates of 60 particles: a pair at zero separation adds
    nothing to the short-range force or to its adjoint (the oracle skips such
    pairs), with and without softening; everything else matches the oracle
    and no value is inf or NaN."""
    from oracle import pp as o_pp
    rng = np.random.default_rng(61)
    base = ics.uniform(1500, seed=62)
    pos = np.concatenate([base, base[:, :60]], axis=1)
    n = pos.shape[1]
    m = rng.uniform(0.5, 1.5, n) / n
    lam = rng.normal(size=(3, n))
    eps = soft_cells * H
    r_s = 1.25 * H
    r_c = 4.5 * r_s
    ref_f = o_pp.pp_accel(pos, m, 1.0, r_s, r_c, eps, 1.0) * m
    ref_v = adjoint.pp_vjp(pos, m, 1.0, r_s, r_c, eps, lam)
    with plan(GRID, n, precision, softening=eps, adjoint=True) as P:
        F = host(P.pp_force(dev(pos), dev(m)))
        g = host(P.pp_force_vjp(dev(pos), dev(m), dev(lam)))
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(g))
    assert _err(F, ref_f) <= (1e-12 if precision == "fp64" else 1e-5)
    assert _err(g, ref_v) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
@pytest.mark.parametrize("fd_order,deconv_power", [(2, 2), (4, 0)])
def test_pm_vjp_gradient_order_and_deconvolution(case, precision, tol, fd_order, deconv_power):
    """The mesh adjoint with the plan's other options (2-point gradient, no
    CIC deconvolution) against the oracle's transpose of the same force."""
    pos, m, lam, _, _ = case
    ref = adjoint.pm_vjp(pos, m, 1.0, GRID, 1.25 * H, lam, fd_order=fd_order,
                         deconv_power=deconv_power)
    with _vjp_plan(pos.shape[1], precision, fd_order=fd_order, deconv_power=deconv_power) as P:
        got = host(P.pm_force_vjp(dev(pos), dev(m), dev(lam)))
    assert _err(got, ref) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_force_vjp_uniform_mass_and_invariants(case, precision):
    """Scalar mass (the per-pair mass factor folded out), and conservation:
    a uniform cotangent has a zero adjoint (total momentum is conserved by
    both force parts)."""
    pos, _, lam, _, _ = case
    n = pos.shape[1]
    ms = 1.0 / n
    ref = adjoint.p3m_vjp(pos, ms, 1.0, GRID, lam, 1.25, 4.5, EPS)
    with _vjp_plan(n, precision) as P:
        x = dev(pos)
        got = host(P.force_vjp(x, ms, dev(lam)))
        uni = np.tile(np.array([[0.7], [-0.2], [1.1]]), (1, n))
        zero = host(P.force_vjp(x, ms, dev(uni)))
    assert _err(got, ref) <= (1e-9 if precision == "fp64" else 1e-4)
    scale = np.sqrt(np.mean(np.sum(ref * ref, axis=0)))
    assert np.sqrt(np.mean(np.sum(zero * zero, axis=0))) <= (1e-9 if precision == "fp64"
                                                             else 1e-4) * scale


def test_force_vjp_matches_gpu_finite_differences(case):
    """<mu, VJP(lam)> against <lam, (F(x + d mu) - F(x - d mu)) / 2d> with the
    GPU's FP64 force: the adjoint is the transpose of the force it ships with."""
    pos, m, lam, _, _ = case
    rng = np.random.default_rng(43)
    mu = rng.normal(size=pos.shape)
    d = 1e-7 * H
    with _vjp_plan(pos.shape[1], "fp64") as P:
        mm = dev(m)
        vjp = host(P.force_vjp(dev(pos), mm, dev(lam)))
        fp = host(P.force(dev((pos + d * mu) % 1.0), mm))
        fm = host(P.force(dev((pos - d * mu) % 1.0), mm))
    lhs = np.sum(mu * vjp)
    rhs = np.sum(lam * (fp - fm)) / (2 * d)
    # pairs crossing r_c or particles crossing node planes within d are rare
    # and each moves the finite difference by a bounded jump
    assert abs(lhs - rhs) <= 1e-4 * np.sum(np.abs(mu * vjp))


def test_drift_vjp_bitwise():
    from paper_1510_07621_amd import binding
    rng = np.random.default_rng(44)
    n = 10007
    xb, pb = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    m = rng.uniform(0.5, 2.0, n)
    dt = 0.0137
    for mass in (m, 0.37):
        zero_vjp = lambda x, l: np.zeros_like(l)
        _, ref = adjoint.leapfrog_vjp([xb, xb], mass, zero_vjp, dt, xb, pb)
        p = dev(pb)
        binding.drift_vjp(p, dev(xb), dev(mass) if isinstance(mass, np.ndarray) else mass, dt)
        np.testing.assert_array_equal(host(p), ref)


def test_vjp_needs_an_adjoint_plan_and_checks_arguments():
    from paper_1510_07621_amd import binding
    pos = dev(ics.uniform(100, seed=45))
    lam = torch.zeros_like(pos)
    with plan(GRID, 100, "fp64") as P:
        with pytest.raises(ValueError):
            P.force_vjp(pos, 0.01, lam)
    with _vjp_plan(100, "fp64") as P:
        with pytest.raises(ValueError):
            P.force_vjp(pos, 0.01, lam, out=pos)            # overlaps pos
        with pytest.raises(ValueError):
            P.force_vjp(pos, 0.01, lam[:, :50].contiguous())
        empty = torch.empty((3, 0), dtype=torch.float64, device="cuda")
        assert P.force_vjp(empty, 0.01, empty).shape == (3, 0)
    with pytest.raises(ValueError):
        binding.drift_vjp(lam, lam, 1.0, 0.1)               # in place on itself


def test_autograd_force_matches_force_vjp(case):
    from paper_1510_07621_amd import autodiff
    pos, m, lam, pp, pm = case
    with _vjp_plan(pos.shape[1], "fp64") as P:
        x = dev(pos).requires_grad_(True)
        F = autodiff.force(P, x, dev(m))
        (g,) = torch.autograd.grad((F * dev(lam)).sum(), x)
    assert _err(host(g), pp + pm) <= 1e-9


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-3)])
@pytest.mark.parametrize("segment", [None, 1, 6])
def test_leapfrog_gradient_matches_the_oracle(precision, tol, segment):
    """6 KDK steps (dt = 0.02) of 1000 particles on a 16^3 grid from small
    random momenta: torch.autograd through autodiff.leapfrog against the
    oracle's transposed trajectory (oracle forward, oracle adjoint), for
    checkpoint segments of ceil(sqrt(6)) = 3 steps, 1 (every state kept) and
    6 (one checkpoint)."""
    from oracle.p3m import p3m_accel
    from paper_1510_07621_amd import autodiff
    rng = np.random.default_rng(46)
    n, steps, dt = 1000, 6, 0.02
    pos = ics.uniform(n, seed=47)
    mom = rng.normal(size=(3, n)) * 1e-4
    ms = 1.0 / n
    xb, pb = rng.normal(size=(3, n)), rng.normal(size=(3, n))

    def force(x):
        return ms * p3m_accel(x, ms, 1.0, GRID, 1.25, 4.5, EPS)

    vjp_fn = lambda x, l: adjoint.p3m_vjp(x, ms, 1.0, GRID, l, **KW)
    xs, pT = adjoint.leapfrog(pos, mom, ms, force, dt, 1.0, steps)
    x0b, p0b = adjoint.leapfrog_vjp(xs, ms, vjp_fn, dt, xb, pb)

    with _vjp_plan(n, precision) as P:
        x0 = dev(pos).requires_grad_(True)
        p0 = dev(mom).requires_grad_(True)
        xT, pT_gpu = autodiff.leapfrog(P, x0, p0, ms, dt, 1.0, steps, segment)
        loss = (xT * dev(xb)).sum() + (pT_gpu * dev(pb)).sum()
        gx, gp = torch.autograd.grad(loss, (x0, p0))
    assert _err(host(xT), xs[-1]) <= 1e-12 * 10 ** (6 if precision == "fp32" else 0)
    assert _err(host(gx), x0b) <= tol
    assert _err(host(gp), p0b) <= tol


def test_zeldovich64_kdk_gradient_matches_finite_differences():
    """The differentiable-KDK workload at full size: 64^3 Zel'dovich ICs, 64^3
    grid, 10 KDK steps of dt = 0.01 from rest, FP64; loss = sum of squared
    final displacements (minimum image, from the initial positions). dL/dx0
    from torch.autograd through autodiff.leapfrog (segments of
    ceil(sqrt(10)) = 4 steps) against central differences of the GPU's own
    trajectory, one particle coordinate at a time (d = 1e-7 box), for 16
    sampled particles x 3 axes. The truncated force jumps where a pair
    crosses r_c, so a difference whose two trajectories do not have the same
    pair count at every step is not a derivative and is left out (at most a
    few); the rest agree to 1e-3 in the norm over the sampled components."""
    from paper_1510_07621_amd import autodiff, binding
    w = ics.workload("zeldovich64_kdk")
    x0 = dev(w.positions())
    p0 = torch.zeros_like(x0)
    with plan(w.grid_n, w.n, "fp64", box=w.box, rs_cells=w.rs_cells, cutoff_rs=w.cutoff_rs,
              softening=w.softening, G=w.G, adjoint=True) as P:

        def loss_of(xT):
            d = xT - x0
            d = d - w.box * torch.round(d / w.box)
            return d

        x = x0.clone().requires_grad_(True)
        xT, _ = autodiff.leapfrog(P, x, p0, w.mass, w.dt, w.box, w.steps)
        dT = loss_of(xT)
        (g,) = torch.autograd.grad((dT * dT).sum(), x)
        g = g.cpu().numpy()

        def trajectory(xs):
            x = xs.clone()
            p = torch.zeros_like(x)
            F = P.force(x, w.mass)
            counts = []
            for _ in range(w.steps):
                binding.kick(p, F, 0.5 * w.dt)
                binding.drift(x, p, w.mass, w.dt, w.box)
                counts.append(P.pair_count(x))
                P.force(x, w.mass, out=F)
                binding.kick(p, F, 0.5 * w.dt)
            return loss_of(x), counts

        rng = np.random.default_rng(48)
        picks = rng.choice(w.n, size=16, replace=False)
        d = 1e-7 * w.box
        fd, ad = [], []
        for k in picks:
            for ax in range(3):
                xp = x0.clone()
                xm = x0.clone()
                xp[ax, k] += d
                xm[ax, k] -= d
                dp, cp = trajectory(xp)
                dm, cm = trajectory(xm)
                if cp != cm:
                    continue
                dl = float(((dp - dm) * (dp + dm)).sum()) / (2 * d)
                fd.append(dl)
                ad.append(g[ax, k])
    fd, ad = np.array(fd), np.array(ad)
    assert len(fd) >= 40
    assert np.linalg.norm(fd - ad) <= 1e-3 * np.linalg.norm(ad)


@pytest.mark.parametrize("name,precision,tol", [
    ("zeldovich64_kdk", "fp64", 1e-11), ("plummer128_kdk", "fp64", 1e-11),
    ("plummer128_kdk", "fp32", 1e-4)])
def test_full_size_force_vjp_sampled(name, precision, tol):
    """The force adjoint at the full sizes of the two adjoint workloads, in
    the plan configuration the bench times, against the oracle's transpose
    on 384 sampled particles (short range from each sample's own pairs, long
    range from the full-grid solve)."""
    from oracle import adjoint as o_adj
    from paper_1510_07621_amd import binding
    w = ics.workload(name)
    pos = w.positions()
    lam = np.random.default_rng(81).normal(size=(3, w.n))
    tg = np.sort(np.random.default_rng(82).choice(w.n, size=384, replace=False))
    ref = (o_adj.pp_vjp(pos, w.mass, w.box, w.r_s, w.r_c, w.softening, lam, w.G, targets=tg) +
           o_adj.pm_vjp(pos, w.mass, w.box, w.grid_n, w.r_s, lam, w.G)[:, tg])
    with binding.Plan(binding.Params(grid_n=w.grid_n, box=w.box, rs_cells=w.rs_cells,
                                     cutoff_rs=w.cutoff_rs, softening=w.softening, G=w.G,
                                     precision=precision, adjoint=1), w.n) as P:
        got = host(P.force_vjp(dev(pos), w.mass, dev(lam)))[:, tg]
    e = _err(got, ref)
    print(name, precision, e)
    assert e <= tol


def _golden_gradient(dt):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        f"plummer16_kdk_grad_dt{dt:g}.txt")
    meta = {}
    with open(path) as f:
        for line in f:
            if not line.startswith("#"):
                break
            parts = line[1:].split()
            if len(parts) == 2 and parts[0] in ("loss", "tangent_norm_growth",
                                                "grad_change_at_1e-12"):
                meta[parts[0]] = float(parts[1])
    return np.loadtxt(path).T, meta


@pytest.mark.parametrize("dt,precision,loss_tol,grad_tol", [
    (0.001, "fp64", 1e-12, 1e-9), (0.001, "fp32", 1e-6, 1e-3),
    (0.01, "fp64", 1e-4, None), (0.01, "fp32", 2e-2, None)])
def test_plummer16_kdk_gradient_against_the_cpu_reference(dt, precision, loss_tol, grad_tol):
    """The clustered differentiable-leapfrog recipe at 16^3 particles: Plummer
    mix (seed 5), 16^3 grid, 50 KDK steps from rest, loss = sum of squared
    final displacements, dL/dx0 from torch.autograd through
    autodiff.leapfrog (checkpoint segments of ceil(sqrt(50)) = 8 steps; FP64
    kick and drift, pair arithmetic in the plan's precision) against the
    oracle's FP64 transposed trajectory stored under tests/golden (written by
    make_plummer16_kdk_gradient.py from the oracle alone).

    dt = 0.001: the trajectory is tame (tangent-norm growth 1.5) and the
    oracle's gradient moves by 7e-11 when x0 moves by 1e-12 of the box; the
    gradient is compared in relative norm (measured FP64 1.2e-11, FP32
    3.6e-5). dt = 0.01: the run is chaotic (tangent-norm growth 7.9e6) and
    the oracle's own gradient changes by a factor of about 28 under that
    1e-12 move, so no precision reproduces it: only the loss is compared
    (measured FP64 1.6e-6, FP32 4e-4 to 2e-3) and the gradient must be
    finite."""
    from paper_1510_07621_amd import autodiff
    ref, meta = _golden_gradient(dt)
    n, steps = 16 ** 3, 50
    pos = ics.plummer_mix(n, 1.0, seed=5)
    ms = 1.0 / n
    with _vjp_plan(n, precision) as P:
        x0 = dev(pos)
        x = x0.clone().requires_grad_(True)
        xT, _ = autodiff.leapfrog(P, x, torch.zeros_like(x0), ms, dt, 1.0, steps, 8)
        d = xT - x                    # displacement from the initial positions themselves
        d = d - torch.round(d)
        loss = (d * d).sum()
        (g,) = torch.autograd.grad(loss, x)
    g = host(g)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    loss_rel = abs(float(loss.detach()) - meta["loss"]) / meta["loss"]
    print(f"plummer16 dt={dt:g} {precision}: grad rel err {rel:.3e}, loss rel err "
          f"{loss_rel:.3e}, oracle tangent-norm growth {meta['tangent_norm_growth']:.4g}, "
          f"oracle gradient change at 1e-12 {meta['grad_change_at_1e-12']:.3g}")
    assert loss_rel <= loss_tol
    assert np.isfinite(g).all()
    if grad_tol is None:
        assert meta["grad_change_at_1e-12"] > 1.0      # ill-conditioned: nothing to match
    else:
        assert meta["grad_change_at_1e-12"] < 1e-9
        assert rel <= grad_tol
