"""The surrogate's training step captured into a HIP graph and replayed
equals the eager loop bit for bit: parameters, Adam moments, step count and
per-epoch losses, over several epochs of replays with eager work (batch
index copies, schedule updates, loss reads) and synchronizations between
them, and again when training resumes with a new graph."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_graph_training_equals_eager(sfg):
    import torch
    from paper_1003_3684_amd import surrogate as sg
    rng = np.random.default_rng(4)
    X = rng.uniform(size=(1024, sg.D_IN)).astype(np.float32)
    Y = rng.normal(size=(1024, sg.D_OUT)).astype(np.float32)
    M = (rng.uniform(size=Y.shape) < 0.9).astype(np.float32)
    eager, graphed = sg.Surrogate(batch=128, seed=2), sg.Surrogate(batch=128, seed=2)
    he = eager.fit(X, Y, M, epochs=4, lr=2e-3, graph=False)
    hg = graphed.fit(X, Y, M, epochs=4, lr=2e-3, graph=True)
    torch.cuda.synchronize()
    assert sfg.device_error() == 0
    assert he == hg and he[-1] < he[0]
    assert eager.step == graphed.step == 4 * 8
    for a, b in ((eager.params, graphed.params), (eager.m, graphed.m), (eager.v, graphed.v)):
        assert torch.equal(a, b)
    he2 = eager.fit(X, Y, M, epochs=2, lr=1e-3, seed=1, graph=False)
    hg2 = graphed.fit(X, Y, M, epochs=2, lr=1e-3, seed=1, graph=True)
    assert he2 == hg2 and eager.step == graphed.step == 6 * 8
    assert torch.equal(eager.params, graphed.params)
    np.testing.assert_array_equal(eager.predict(X[:256]), graphed.predict(X[:256]))
