"""The surrogate trained on generated graphs: its predictions track the
generator, and inverting it reaches target exponents with fewer generator
runs than the same search without it (the generator judges every answer)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    from paper_1003_3684_amd import surrogate as sg
    rng = np.random.default_rng(11)
    k = 12
    rows = [sg.kron_row(a, b, k, 31, graph_id=i) for i, (a, b) in enumerate(rng.uniform(0.03, 0.97, size=(3072, 2)))]
    Y, M = sg.generate_dataset(rows, samples=2000, stat_seed=5, max_batch_edges=1 << 26)
    X = sg.features(rows)
    model = sg.Surrogate(batch=128, seed=1)
    hist = model.fit(X[:2560], Y[:2560], M[:2560], epochs=100, lr=2e-3)
    return sg, model, X, Y, M, hist, k


def test_training_converges(trained):
    sg, model, X, Y, M, hist, k = trained
    assert hist[-1] < 0.2 * hist[0], hist[:3] + hist[-3:]


def test_heldout_gamma_prediction(trained):
    # Held-out graphs: over the middle 60% of exponents the median error of
    # the prediction is a small fraction of that range's width.
    sg, model, X, Y, M, hist, k = trained
    pred = sg.Surrogate.gamma_of(model.predict(X[2560:]))
    ok = M[2560:, sg.GAMMA_COL] > 0
    y = sg.Surrogate.gamma_of(Y[2560:])[ok]
    err = np.abs(pred[ok] - y)
    lo, hi = np.quantile(y, [0.2, 0.8])
    mid = (y > lo) & (y < hi)
    assert np.median(err[mid]) < 0.05 * (hi - lo), (np.median(err[mid]), lo, hi)


def test_inversion_beats_generator_only_search(trained):
    sg, model, X, Y, M, hist, k = trained
    # Exponents of the usual scale-free range, all inside the training data.
    g = sg.Surrogate.gamma_of(Y)[M[:, sg.GAMMA_COL] > 0]
    targets = np.array([2.2, 2.5, 2.8, 3.1])
    assert g.min() < targets.min() and targets.max() < g.max()
    judge = sg.Judge(k=k, seeds=(31,), samples=2000)
    tol = 0.05
    with_s, without = [], []
    for i, t in enumerate(targets):
        ok1, c1 = sg.search_with_surrogate(model, judge, float(t), tol, budget=40, seed=i)
        ok2, c2 = sg.search_generator_only(judge, float(t), tol, budget=40, seed=i)
        with_s.append(c1 if ok1 else 41)
        without.append(c2 if ok2 else 41)
    print("generator runs with surrogate", with_s, "without", without)
    assert np.mean(with_s) < np.mean(without)
