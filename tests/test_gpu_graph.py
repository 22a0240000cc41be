"""Time steps replayed from a captured HIP graph (SD.rk_steps with
graph_steps > 0) against the same steps launched one by one: the graph holds
the same kernels on the same buffers, so the states agree bit for bit.  The
graph is replayed in several calls, with the program's own eager work and
synchronising calls (diagnostics, host copies) between them, and every
replay's state is checked."""
import math

import numpy as np
import pytest

from paper_2608_09615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def pair(torch, make, U0, dt, rounds, graph_steps, between=None):
    """The eager and the graph-replayed runs of `rounds` calls of
    graph_steps + 1 steps each; returns the largest difference per round."""
    from paper_2608_09615_amd import SD  # noqa: F401
    a, b = make(), make()
    ua = torch.from_numpy(U0.copy()).to("cuda")
    ub = torch.from_numpy(U0.copy()).to("cuda")
    out = []
    for _ in range(rounds):
        for _ in range(graph_steps + 1):
            a.rk_step(ua, dt)
        b.rk_steps(ub, dt, graph_steps + 1, graph_steps=graph_steps)
        if between is not None:
            between(b, ub)
        torch.cuda.synchronize()
        out.append(float(np.abs(ua.cpu().numpy() - ub.cpu().numpy()).max()))
    assert len(b._graphs) == 1           # one capture, replayed in every round
    a.close()
    b.close()
    return out


def test_graph_steps_1d_diffusion(torch_cuda):
    from paper_2608_09615_amd import SD
    N, p = 16, 3
    x = W.points_1d(N, p, 0.0, 2 * math.pi)
    U0 = np.ascontiguousarray(np.sin(x)[:, None, :])
    h = 2 * math.pi / N
    dt = 0.05 * h * h / (p + 1) ** 2
    make = lambda: SD([N], p, scheme="compact", physics="diffusion", precision="fp64", lo=[0.0], hi=[2 * math.pi])
    d = pair(torch_cuda, make, U0, dt, rounds=4, graph_steps=16)
    print("1-D diffusion:", d)
    assert max(d) == 0.0


@pytest.mark.parametrize("precision,integrator", [("fp32", "rk4"), ("fp64", "rk4"), ("fp64", "ssprk54"),
                                                  ("bf16x3", "rk4")])
def test_graph_steps_navier_stokes(torch_cuda, precision, integrator):
    """The chained FP32 stages (the stage state in compute precision, two
    alternating buffers), FP64, the SSP scheme's separate combinations, and
    BF16x3; diagnostics (a host-synchronising call) between the replays."""
    from paper_2608_09615_amd import SD
    nel, p = (4, 3, 5), 3
    lo, hi = W.tgv_domain()
    U0 = W.perturbed_tgv_state(nel, p, seed=3, noise=1e-3)
    make = lambda: SD(nel, p, scheme="compact", physics="ns", precision=precision, lo=lo, hi=hi,
                      integrator=integrator)
    d = pair(torch_cuda, make, U0, 2e-3, rounds=3, graph_steps=5, between=lambda sd, u: sd.diagnostics(u))
    print(f"NS {precision} {integrator}:", d)
    assert max(d) == 0.0


def test_graph_steps_curvilinear(torch_cuda):
    from paper_2608_09615_amd import SD
    nel, p = (3, 2, 4), 3
    Xg = W.mesh_nodes(nel, (0.0, 0.0, 0.0), (2 * math.pi,) * 3, q=2,
                      displacement=W.periodic_wave_displacement(0.2))
    lo, hi = W.tgv_domain()
    U0 = W.perturbed_tgv_state(nel, p, seed=5, noise=1e-2)

    def make():
        sd = SD(nel, p, scheme="compact", physics="ns", precision="fp32", lo=lo, hi=hi)
        sd.set_geometry(Xg)
        return sd
    d = pair(torch_cuda, make, U0, 1e-3, rounds=3, graph_steps=4)
    print("curvilinear NS fp32:", d)
    assert max(d) == 0.0
