"""The force path under HIP graph capture: a captured force call (its
second-stream fork and join included) and a captured KDK step replay to the
eager results, with eager work between the replays."""
import numpy as np
import pytest
import torch

from paper_1510_07621_amd import ics

from _gpu import dev, host, plan, require_gpu

pytestmark = pytest.mark.gpu


def _max_rel(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=0)) / np.max(np.linalg.norm(b, axis=0)))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_force_call_replays_in_a_graph(precision, tol):
    require_gpu()
    n = 8000
    pos = ics.uniform(n, seed=71)
    with plan(32, n, precision, softening=1e-3) as P:
        x = dev(pos)
        want = host(P.force(x, 1.0 / n))
        F = torch.empty_like(x)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            P.force(x, 1.0 / n, out=F)           # warm-up on the capture's kind of stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            P.force(x, 1.0 / n, out=F)
        for _ in range(3):
            F.fill_(7.0)                          # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            assert _max_rel(host(F), want) < tol


def test_kdk_step_replays_in_a_graph():
    """Three replays of a captured step (fused kick + drift, force, kick)
    against three eager steps from the same state, FP64."""
    require_gpu()
    from paper_1510_07621_amd import binding
    n, dt = 8000, 0.002
    pos = ics.uniform(n, seed=72)
    mom = np.random.default_rng(73).normal(size=(3, n)) * 1e-3
    m = 1.0 / n
    with plan(32, n, "fp64", softening=1e-3) as P:
        # eager reference
        xe, pe = dev(pos), dev(mom)
        Fe = P.force(xe, m)
        for _ in range(3):
            binding.kick_drift(xe, pe, Fe, m, 0.5 * dt, dt, 1.0)
            P.force(xe, m, out=Fe)
            binding.kick(pe, Fe, 0.5 * dt)
        x_want, p_want = host(xe), host(pe)
        # captured step
        x, p = dev(pos), dev(mom)
        F = P.force(x, m)
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        xs, ps, Fs = x.clone(), p.clone(), F.clone()
        with torch.cuda.stream(side):             # warm-up step on copies
            binding.kick_drift(xs, ps, Fs, m, 0.5 * dt, dt, 1.0)
            P.force(xs, m, out=Fs)
            binding.kick(ps, Fs, 0.5 * dt)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            binding.kick_drift(x, p, F, m, 0.5 * dt, dt, 1.0)
            P.force(x, m, out=F)
            binding.kick(p, F, 0.5 * dt)
        for _ in range(3):
            torch.cuda.synchronize()
            g.replay()
        assert _max_rel(host(x), x_want) < 1e-12
        assert _max_rel(host(p), p_want) < 1e-9
