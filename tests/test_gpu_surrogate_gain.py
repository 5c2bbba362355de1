"""What the trained surrogate gains over plain RK4, end to end on the GPU.

Trajectories come from the library's own batched integrator (2D defocusing
NLSE, 256^2, 2SHOC + MSD, compensated FP32); the network is trained on them
by the library's forward / backward / Adam kernels; held-out trajectories
then measure (a) the one-block error against 16 RK4 steps, next to the error
of not advancing at all, (b) the time of one surrogate block against 16 RK4
steps at the same batch, and (c) the guarded advance, whose mass check sends
blocks back to RK4.

The training here is short (seconds), so the accuracy bound is looser than
the full run's (0.8% after 3000 iterations on 20 000 pairs): 2e-2 relative
L2, and at most a quarter of the do-nothing error.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_1263_amd import surrogate_train as st
    snaps = st.generate(28, npairs=24, burn=160, seed_index=11)
    train_idx = np.arange(24)
    m, params, hist, secs = st.train(snaps, train_idx, iters=500, batch=16, lr=1e-3, seed=3, log_every=250)
    test_idx = torch.arange(24, 28, device="cuda")
    yield st, m, snaps, test_idx, hist
    m.close()


def test_training_converges(trained):
    st, m, snaps, test_idx, hist = trained
    assert hist[-1][1] < 0.05 * hist[0][1]


def test_one_block_error_beats_doing_nothing(trained):
    st, m, snaps, test_idx, _ = trained
    errs, still = [], []
    for k in range(0, snaps.shape[1] - 1, 4):
        x = snaps[test_idx, k].contiguous()
        y = snaps[test_idx, k + 1]
        p = m.forward(x)
        m.project_msd(x, p)
        errs.append(st._rel(p, y))
        still.append(st._rel(x, y))
    err, base = float(np.mean(errs)), float(np.mean(still))
    print(f"one-block rel L2: surrogate {err:.3e}, unchanged field {base:.3e}")
    assert err < 2e-2
    assert err < 0.25 * base


def test_surrogate_block_is_faster_than_16_rk4_steps(trained):
    st, m, snaps, test_idx, _ = trained
    r = st.speedup(m, snaps, 16)
    print(f"batch 16: RK4 {r['ms_rk4_16_steps']:.3f} ms, surrogate {r['ms_surrogate_block']:.3f} ms, "
          f"speedup {r['speedup']:.2f}x, forward {r['forward_tflops']:.0f} TFLOP/s")
    assert r["speedup"] > 1.5


def test_guarded_advance_tracks_rk4(trained):
    st, m, snaps, test_idx, _ = trained
    g = st.guarded_advance(m, snaps, test_idx.tolist()[:2], nblocks=4, tol=1e-3)
    print(g)
    assert g["rel_l2_guarded"] < 0.1
