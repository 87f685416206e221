"""The surrogate's training step captured into a HIP graph and replayed
equals the eager loop bit for bit: parameters, Adam moments, step count and
per-epoch losses, over several epochs of replays with eager work (batch
index copies, schedule updates, loss reads) and synchronizations between
them, and again when training resumes with a new graph -- for the fused
step and for the unfused kernels; and the two train alike."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fused", [True, False])
def test_graph_training_equals_eager(sfg, fused):
    import torch
    from paper_1003_3684_amd import surrogate as sg
    rng = np.random.default_rng(4)
    X = rng.uniform(size=(1024, sg.D_IN)).astype(np.float32)
    Y = rng.normal(size=(1024, sg.D_OUT)).astype(np.float32)
    M = (rng.uniform(size=Y.shape) < 0.9).astype(np.float32)
    eager, graphed = sg.Surrogate(batch=128, seed=2), sg.Surrogate(batch=128, seed=2)
    assert eager.tws is not None
    he = eager.fit(X, Y, M, epochs=4, lr=2e-3, graph=False, fused=fused)
    hg = graphed.fit(X, Y, M, epochs=4, lr=2e-3, graph=True, fused=fused)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    assert he == hg and he[-1] < he[0]
    assert eager.step == graphed.step == 4 * 8
    for a, b in ((eager.params, graphed.params), (eager.m, graphed.m), (eager.v, graphed.v)):
        assert torch.equal(a, b)
    he2 = eager.fit(X, Y, M, epochs=2, lr=1e-3, seed=1, graph=False, fused=fused)
    hg2 = graphed.fit(X, Y, M, epochs=2, lr=1e-3, seed=1, graph=True, fused=fused)
    assert he2 == hg2 and eager.step == graphed.step == 6 * 8
    assert torch.equal(eager.params, graphed.params)
    np.testing.assert_array_equal(eager.predict(X[:256]), graphed.predict(X[:256]))


def test_fused_and_unfused_training_agree(sfg):
    """The same data and schedule through the fused step and through the
    unfused kernels: they differ only in float32 summation order, so the
    per-epoch losses agree closely and both fall."""
    from paper_1003_3684_amd import surrogate as sg
    rng = np.random.default_rng(5)
    X = rng.uniform(size=(2048, sg.D_IN)).astype(np.float32)
    Y = (X[:, :1] * 2 - 1 + 0.1 * rng.normal(size=(2048, sg.D_OUT))).astype(np.float32)
    M = np.ones_like(Y)
    a, b = sg.Surrogate(batch=256, seed=3), sg.Surrogate(batch=256, seed=3)
    ha = a.fit(X, Y, M, epochs=6, lr=2e-3, fused=True)
    hb = b.fit(X, Y, M, epochs=6, lr=2e-3, fused=False)
    assert sfg.device_error() == 0
    assert ha[-1] < 0.5 * ha[0] and hb[-1] < 0.5 * hb[0], (ha, hb)
    np.testing.assert_allclose(ha, hb, rtol=2e-2)
