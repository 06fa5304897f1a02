"""Thm. 5.1 as a run-time precision selector (casgd_select_precision) against
the oracle's evaluation of the same bound (on an MI355X).

The library gathers the sampled block, forms G_L, the margins and the exact
residual history on the GPU and evaluates the theorem's norms on the host
(Lanczos); the oracle evaluates the same quantities with dense FP64 linear
algebra from the exact rows. They agree to the rounding of the GPU's FP32
Gram and margins (relative 1e-5). The choice is the first candidate, in the
documented order, whose relative bound meets the budget.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import dense_c1, dense_glm  # noqa: E402

U32 = 2.0 ** -24
U_OF = {0: 0.0, 1: 2.0 ** -8, 2: 2.0 ** -11, 3: 2.0 ** -4}


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _normalised(X):
    return (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("b,s", [(16, 4), (32, 8), (64, 16), (8, 1)])
@pytest.mark.parametrize("loss", ["logistic", "linear", "poisson"])
def test_selector_terms_match_oracle(cg, b, s, loss):
    if loss == "logistic":
        p = dense_c1(42)
        X32 = _normalised(p.X)
        y = p.y.astype(np.float32)
        eta = 0.5
    else:
        p = dense_glm(4096, 256, 5, loss, var=1 / 256)
        X32 = _normalised(p.X)
        y = p.y.astype(np.float32)
        eta = 0.5 if loss == "linear" else 0.2
    x = (np.random.default_rng(3).standard_normal(256) * 0.2).astype(np.float32)
    seed, h = 42, 3
    rep = cg.casgd_select_precision(cg.dense_matrix(_dev(X32)), _dev(y), _dev(x), eta, b, s, seed,
                                    h, loss=loss, rel_budget=1e-3)
    idx = R.sample_indices(seed, h * s * b, s * b, X32.shape[0])
    Y = X32[idx].astype(np.float64)
    yI = y[idx].astype(np.float64)
    L_sigma = {"logistic": 0.25, "linear": 1.0}.get(loss)
    if loss == "poisson":
        L_sigma = rep["L_sigma"]
        # the Poisson constant is exp(max z) over the block of the exact recurrence
        o0 = R.local_error_bound(Y, x, yI, b, s, eta, u_A=0, gamma_r=0, gamma_G=0, u_c=0,
                                 u_sigma=0, gamma_g=0, u_x=0, loss=loss)
        G = Y @ Y.T * R.strict_block_lower_mask(b, s)
        z = Y @ x.astype(np.float64) + (eta / b) * (G @ o0["d"])
        assert rep["L_sigma"] == pytest.approx(float(np.exp(z.max())), rel=1e-5)
    D_delta = rep["D_delta"] if loss != "logistic" else 1.0
    for c in rep["candidates"]:
        u = c["u"]
        o = R.local_error_bound(Y, x, yI, b, s, eta, u_A=u["A"], gamma_r=u["r"],
                                gamma_G=u["G"], u_c=u["c"], u_sigma=u["sigma"], gamma_g=u["g"],
                                u_x=u["x"], L_sigma=L_sigma, D_delta=D_delta, loss=loss)
        for q, key in (("A", "A"), ("r", "r"), ("G", "G"), ("c", "c"), ("sigma", "sigma"),
                       ("g", "g"), ("x", "x")):
            assert c["E"][q] == pytest.approx(o["E"][key], rel=1e-5, abs=1e-300), (c["dtype"], q)
        assert c["sum"] == pytest.approx(o["sum"], rel=1e-5)
        assert c["Omega"] == pytest.approx(o["Omega"], rel=1e-5)
        assert c["bound"] == pytest.approx(o["bound"], rel=1e-5)
    o = R.local_error_bound(Y, x, yI, b, s, eta, u_A=0, gamma_r=0, gamma_G=0, u_c=0,
                            u_sigma=0, gamma_g=0, u_x=0, L_sigma=L_sigma, D_delta=D_delta,
                            loss=loss)
    for name in ("norm_Y", "norm_HL", "T_g", "T_r", "T_G", "T_c"):
        assert rep[name] == pytest.approx(o[name], rel=1e-5, abs=1e-300), name
    assert rep["K_s"] == pytest.approx(o["K_s"], rel=1e-5)


def test_selector_choice_follows_the_budget(cg):
    p = dense_c1(42)
    X32 = _normalised(p.X)
    Xd = cg.dense_matrix(_dev(X32))
    y, x = _dev(p.y.astype(np.float32)), _dev(np.zeros(256, np.float32))
    b, s, eta = 32, 8, 0.5
    order = [3, 1, 2, 0]
    seen = []
    for budget in (1.0, 1e-2, 1e-4, 1e-6, 1e-9, 1e-30):
        rep = cg.casgd_select_precision(Xd, y, x, eta, b, s, 42, 0, rel_budget=budget)
        cands = rep["candidates"]
        # candidates in the documented order: storage cheapest first, FP32
        # corrections before FP64
        assert [c["dtype"] for c in cands] == [d for d in order for _ in range(2)]
        assert [c["recur_prec"] for c in cands] == [32, 64] * 4
        ok = [i for i, c in enumerate(cands) if c["valid"] and c["rel_bound"] <= budget]
        if ok:
            assert rep["meets_budget"] and rep["chosen"] == ok[0]
        else:
            assert not rep["meets_budget"]
            assert rep["chosen"] == max(i for i, c in enumerate(cands) if c["valid"])
        assert rep["dtype"] == cands[rep["chosen"]]["dtype"]
        seen.append((rep["dtype"], rep["recur_prec"]))
        # a bound grows with every slot's unit roundoff
        assert all(c["u"]["A"] == U_OF[c["dtype"]] for c in cands)
    # a loose budget admits low-precision storage (here BF16: the FP8 bound
    # exceeds ||x^(s)||), the tightest one only FP32
    print("\n[selector] rel bounds:", [(c["dtype"], c["recur_prec"], f"{c['rel_bound']:.2e}",
                                         c["valid"]) for c in cands])
    assert seen[0][0] != 0 and seen[-1][0] == 0
    # restricting the allowed formats
    rep = cg.casgd_select_precision(Xd, y, x, eta, b, s, 42, 0, rel_budget=1.0,
                                    allowed=(1 << 1) | (1 << 0))
    assert rep["dtype"] == 1


def test_selector_rejects_bad_arguments(cg):
    p = dense_c1(42)
    X32 = p.X.astype(np.float32)
    v, _ = cg.casgd_quantize(_dev(X32), cg.BF16)
    with pytest.raises(cg.CasgdError):
        cg.casgd_select_precision(cg.dense_matrix(v, None, n=256), _dev(p.y), _dev(np.zeros(256,
                                  np.float32)), 0.5, 16, 4, 1)
    with pytest.raises(cg.CasgdError):
        cg.casgd_select_precision(cg.dense_matrix(_dev(X32)), _dev(p.y),
                                  _dev(np.zeros(256, np.float32)), 0.5, 16, 4, 1, rel_budget=0.0)
