"""Learned diagonal preconditioner end to end on small uneven problems: targets
from plain runs, MLP training with the library's kernels, prediction on unseen
problems, and the preconditioned fit against the plain one."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import uneven_problem, uneven_problem_specs  # noqa: E402

pytestmark = pytest.mark.gpu

LAM, B, S, SEED = 1e-5, 16, 4, 11


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2606_18463_amd import learned
    return learned


def _problems(count, seed):
    specs = uneven_problem_specs(count, seed, m_range=(3000, 6000), n_range=(64, 256),
                                 spread_range=(3.0, 300.0))
    return [uneven_problem(sp) for sp in specs]


def test_learned_preconditioner_generalises(L):
    train_p = [L.upload(p, dtype=0) for p in _problems(12, 1)]
    test_p = [L.upload(p, dtype=0) for p in _problems(4, 2)]
    stats, tds, tetas = [], [], []
    for dp in train_p:
        t_d, log_eta, _ = L.targets(dp, LAM, B, S, SEED, epochs=1.0)
        stats.append(L.cg.casgd_colstats(L.stored(dp)))
        tds.append(t_d)
        tetas.append(log_eta)
    model, hist = L.train(stats, tds, tetas, steps=400, lr=1e-2, log_every=100)
    print("mlp loss", hist)
    assert hist[-1][1] < 0.5 * hist[0][1]

    corr, wins = [], 0
    for dp in test_p:
        X = L.stored(dp)
        Xq, _, q, eta = L.apply(model, dp)
        # predicted scale against the Jacobi target of the unseen problem
        t_d, _, eta0 = L.targets(dp, LAM, B, S, SEED, epochs=1.0)
        pred = 2.0 * torch.log(q)
        corr.append(float(torch.corrcoef(torch.stack([pred, t_d]))[0, 1]))
        n_outer = max(2, int(dp.m / (B * S)))
        x_plain, _ = L.fit(X, dp.y, dp.n, eta0, LAM, B, S, SEED, n_outer)
        lp = float(L.cg.casgd_logloss(dp.Xt, dp.yt, x_plain))
        xt, _ = L.fit(Xq, dp.y, dp.n, eta, LAM, B, S, SEED, n_outer)
        ll = float(L.cg.casgd_logloss(dp.Xt, dp.yt, L.unscale(xt, q)))
        print("problem", dp.m, dp.n, "plain", lp, "learned", ll, "eta", eta0, eta)
        wins += ll < lp
    print("corr", corr)
    assert min(corr) > 0.5
    assert wins >= 3
