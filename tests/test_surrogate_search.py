"""Host logic of the surrogate-guided search, with a stand-in surrogate
(an analytic u(a, b) = log(gamma - 1)) and a stand-in generator that differs
from it by a smooth offset, so that no GPU is needed: the guided search
reaches each target in a few judged runs, fewer than the random search, and
the fallback takes over when the surrogate is useless."""
import math

import numpy as np

from paper_1003_3684_amd import surrogate as sg


def _u(a, b):
    return np.log(0.25 + 1.5 * (a - b) ** 2 + 0.6 * a)


class MockModel:
    def __init__(self, flat=False):
        self.flat = flat

    def log_tail_and_grad(self, X):
        a, b = X[:, 5].astype(np.float64), X[:, 7].astype(np.float64)
        inner = 0.25 + 1.5 * (a - b) ** 2 + 0.6 * a
        dX = np.zeros((len(X), X.shape[1]))
        if self.flat:  # a useless surrogate: constant prediction, no gradient
            return np.zeros(len(X)), dX
        dX[:, 5] = (3.0 * (a - b) + 0.6) / inner
        dX[:, 7] = -3.0 * (a - b) / inner
        return np.log(inner), dX

    def gamma_and_grad(self, X):
        u, du = self.log_tail_and_grad(X)
        return 1.0 + np.exp(u), du * np.exp(u)[:, None]


class MockJudge:
    """The 'generator': the surrogate's u plus a smooth offset."""

    def __init__(self, k=12):
        self.k, self.calls = k, 0

    def gamma(self, a, b):
        self.calls += 1
        return 1.0 + math.exp(_u(a, b) + 0.12 + 0.15 * a - 0.1 * b)


def test_guided_search_beats_random_search():
    targets = [1.6, 1.9, 2.2, 2.5]
    guided, random_ = [], []
    for i, t in enumerate(targets):
        ok, c = sg.search_with_surrogate(MockModel(), MockJudge(), t, 0.01, budget=40, seed=i)
        assert ok, (t, c)
        guided.append(c)
        ok2, c2 = sg.search_generator_only(MockJudge(), t, 0.01, budget=40, seed=i)
        random_.append(c2 if ok2 else 41)
    assert max(guided) <= 6, guided
    assert np.mean(guided) < np.mean(random_), (guided, random_)


def test_fallback_to_generator_only():
    # A useless surrogate and a tolerance no start meets: the surrogate's
    # share of the budget is spent, the generator-only search spends the
    # rest, and every call is counted once.
    judge = MockJudge()
    ok, calls, which = sg.fit_exponent(MockModel(flat=True), judge, 1.9, 1e-5, budget=20, seed=3)
    assert not ok and which == "generator" and calls == judge.calls == 20
    ok, calls, which = sg.fit_exponent(MockModel(), MockJudge(), 1.9, 0.01, budget=40, seed=3)
    assert ok and which == "surrogate" and calls <= 6
