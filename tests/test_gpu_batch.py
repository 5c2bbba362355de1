"""GPU tests of the batched persistent integrator (many 2D problems in one
launch).  Bar: FP32 relative L2 <= 1e-5 against the FP64 oracle per problem;
a problem inside a batch is bitwise equal to the same problem run alone; every
replay of the captured graph is bitwise equal to the direct launch."""
import os

import numpy as np
import pytest

import oracle
from paper_1203_1263_amd import workloads as wl
from gpu_util import rel_l2

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class P:  # minimal problem record
    def __init__(self, psi0, h, a, s, V, order, bc):
        self.psi0, self.h, self.a, self.s, self.V, self.order, self.bc = psi0, h, a, s, V, order, bc


SHAPES = [(37, 70), (64, 64), (3, 3), (45, 100), (9, 130), (8, 32), (70, 37), (5, 5), (33, 65), (16, 200),
          (100, 9), (31, 33)]


def small_batch(seed=5):
    g = np.random.default_rng(seed)
    probs, dts = [], []
    for k, (ny, nx) in enumerate(SHAPES):
        # modulus in ~[0.5, 2]; weak focusing only, so no problem collapses
        u = 1.2 + 0.25 * wl.random_field((ny, nx), 300 + k, smooth=2.0)
        V = 0.3 * wl.random_field((ny, nx), 300 + k, stream=1, smooth=3.0).real if k % 3 else None
        order = (2, 4)[k % 2]
        bc = ("dirichlet", "msd", "l0")[(k // 2) % 3]
        h, a, s = float(g.uniform(0.2, 0.4)), float(g.uniform(0.5, 1.0)), float(g.choice([-1.0, 0.2]))
        probs.append(P(u, h, a, s, V, order, bc))
        dts.append(0.5 * oracle.dt_max(2, order, h, a))
    return probs, dts


@pytest.mark.parametrize("dtype,comp,graph", [("f32", True, True), ("f32", False, True), ("f64", False, True),
                                              ("f32", True, False)])
def test_batch_matches_oracle_and_single_grid(dtype, comp, graph):
    import torch
    from paper_1203_1263_amd.nlse import Batch, Grid
    from gpu_util import to_dev, pot_dev
    probs, dts = small_batch()
    n = 10
    b = Batch(probs, dts, dtype=dtype, compensated=comp, graph=graph)
    b.step(n)
    b.status()
    torch.cuda.synchronize()
    tol = 1e-5 if dtype == "f32" else 1e-11
    for j, (p, dt) in enumerate(zip(probs, dts)):
        got = b.field(j).cpu().numpy().astype(np.complex128)
        ref = oracle.rk4(p.psi0, p.h, p.a, p.s, dt, n, V=p.V, order=p.order, bc=p.bc)
        assert rel_l2(got, ref) < tol, f"problem {j}"
        psi = to_dev(p.psi0, dtype)
        g = Grid(psi, p.h, p.a, p.s, V=pot_dev(p.V, dtype), compensated=comp)
        g.set_tile(p.order, (32, 8, 1))
        g.step(dt, n, order=p.order, bc=p.bc)
        torch.cuda.synchronize()
        assert torch.equal(psi, b.field(j)), f"problem {j} differs from its single-grid run"
        g.close()
    M, E = b.mass_energy()
    for j, p in enumerate(probs):
        ref = oracle.rk4(p.psi0, p.h, p.a, p.s, dts[j], n, V=p.V, order=p.order, bc=p.bc)
        Mr, Er = oracle.mass_energy(ref, p.h, p.a, p.s, V=p.V, order=p.order, bc=p.bc)
        assert M[j] == pytest.approx(Mr, rel=1e-5 if dtype == "f32" else 1e-11)
    b.close()


def test_graph_replays_match_direct_launches():
    """Three replays of the captured graph, with other device work and
    synchronisations between them, each bitwise equal to direct launches."""
    import torch
    from paper_1203_1263_amd.nlse import Batch
    probs, dts = small_batch(9)
    direct = Batch(probs, dts, compensated=True, graph=False)
    graph = Batch(probs, dts, compensated=True, graph=True)
    scratch = torch.randn(1 << 20, device="cuda")
    for r in range(3):
        direct.step(7)
        graph.step(7)
        scratch.mul_(1.0001).add_(0.5)          # unrelated eager work between replays
        direct.mass_energy()                    # reductions + synchronisation
        torch.cuda.synchronize()
        assert torch.equal(direct.pool, graph.pool), f"replay {r}"
    assert graph.info()["graphs"] == 1
    direct.status()
    graph.status()


def test_barrier_timeout_is_reported_and_the_grid_drains(monkeypatch):
    """A wait at a group barrier that runs out (forced from the host: a spin
    limit of one poll) sets the error flag; the launch still completes,
    nlse_batch_status reports NLSE_EDEVICE, and a later launch of the same
    batch completes too (waiting workgroups leave at once)."""
    import torch
    from paper_1203_1263_amd import nlse
    from paper_1203_1263_amd.nlse import Batch
    probs, dts = small_batch()
    monkeypatch.setenv("NLSE_BATCH_SPIN_LIMIT", "1")
    b = Batch(probs, dts, compensated=True)
    monkeypatch.delenv("NLSE_BATCH_SPIN_LIMIT")
    b.step(5)
    torch.cuda.synchronize()
    with pytest.raises(nlse.NLSEError) as e:
        b.status()
    assert e.value.code == nlse.NLSE_EDEVICE
    b.step(3)
    torch.cuda.synchronize()
    with pytest.raises(nlse.NLSEError):
        b.status()
    # a batch created without the override is unaffected
    b2 = Batch(probs, dts, compensated=True)
    b2.step(5)
    b2.status()


def test_batch_info_and_schedule():
    from paper_1203_1263_amd.nlse import Batch
    probs, dts = small_batch()
    b = Batch(probs, dts)
    info = b.info()
    items = sum(((nx + 31) // 32) * ((ny + 7) // 8) for ny, nx in SHAPES)
    assert info["items"] == items
    assert info["points"] == sum(ny * nx for ny, nx in SHAPES)
    assert 1 <= info["workgroups"] <= items


def test_c4_batch_512_problems_500_steps():
    """The 512-problem workload (uneven sizes 64..512, CD2/2SHOC, a, s, V per
    problem), 500 steps in one launch, sampled against the FP64 oracle."""
    import torch
    from paper_1203_1263_amd.nlse import Batch
    path = os.path.join(GOLDEN, "c4_batch2d_512x500.npz")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    G = np.load(path, allow_pickle=False)
    probs = wl.batch2d()
    dts = [p.dt_fraction * oracle.dt_max(2, p.order, p.h, p.a) for p in probs]
    b = Batch(probs, dts, compensated=True)
    b.step(500)
    b.status()
    torch.cuda.synchronize()
    worst = 0.0
    for j in G["sel"]:
        assert dts[j] == float(G[f"dt{j}"])
        got = b.field(int(j)).reshape(-1).cpu().numpy().astype(np.complex128)
        err = rel_l2(got[G[f"idx{j}"]], G[f"val{j}"])
        worst = max(worst, err)
        assert err < 1e-5, f"problem {j}: {err:.3e}"
    print(f"c4 worst sampled rel L2 {worst:.3e}")
