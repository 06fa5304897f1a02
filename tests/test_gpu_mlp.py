"""Learned-preconditioner kernels vs the FP64 oracle (MI355X)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import dense_logreg  # noqa: E402


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


def _params(g):
    W1 = g.standard_normal((64, 4)) * 0.5
    b1 = g.standard_normal(64) * 0.1
    W2 = g.standard_normal((2, 64)) * 0.3
    b2 = g.standard_normal(2) * 0.1
    flat = np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)
    return flat, [a.astype(np.float32).astype(np.float64) for a in (W1, b1, W2, b2)]


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("N,P", [(1000, 3), (4097, 17), (64, 1)])
def test_mlp_forward_loss_backward_vs_oracle(cg, N, P):
    g = np.random.default_rng(N + P)
    flat, (W1, b1, W2, b2) = _params(g)
    F = g.standard_normal((N, 4)).astype(np.float32)
    cuts = np.sort(g.choice(np.arange(1, N), size=P - 1, replace=False)) if P > 1 else []
    seg_off = np.concatenate([[0], cuts, [N]]).astype(np.int64)
    seg = np.repeat(np.arange(P), np.diff(seg_off))
    t_d = g.standard_normal(N).astype(np.float32)
    t_eta = g.standard_normal(P).astype(np.float32)
    out, pre = cg.casgd_mlp_forward(_dev(flat), _dev(F))
    o_ref, h_ref, pre_ref = R.mlp_forward(F.astype(np.float64), W1, b1, W2, b2)
    assert np.allclose(out.cpu().numpy(), o_ref, rtol=1e-5, atol=1e-5)
    assert np.allclose(pre.cpu().numpy(), pre_ref, rtol=1e-5, atol=1e-5)
    loss, gout = cg.casgd_mlp_loss_grad(out, _dev(seg_off, torch.int64), _dev(t_d), _dev(t_eta),
                                        0.5)
    L_ref, g_ref = R.mlp_loss(out.cpu().numpy().astype(np.float64), seg, t_d.astype(np.float64),
                              t_eta.astype(np.float64), 0.5)
    assert abs(loss.item() - L_ref) <= 1e-9 * max(1.0, abs(L_ref))
    assert np.allclose(gout.cpu().numpy(), g_ref, rtol=1e-5, atol=1e-9)
    grad = cg.casgd_mlp_backward(_dev(flat), _dev(F), pre, gout, P).cpu().numpy()
    gw = R.mlp_backward(F.astype(np.float64), np.maximum(pre.cpu().numpy().astype(np.float64), 0),
                        pre.cpu().numpy().astype(np.float64), W2,
                        gout.cpu().numpy().astype(np.float64))
    ref = np.concatenate([gw[0].ravel(), gw[1], gw[2].ravel(), gw[3]])
    scale = np.abs(ref).max()
    assert np.max(np.abs(grad - ref)) <= 1e-5 * scale + 1e-7


def test_adam_vs_oracle(cg):
    g = np.random.default_rng(3)
    p = g.standard_normal(450).astype(np.float32)
    pd, m1, m2 = _dev(p), torch.zeros(450, device="cuda"), torch.zeros(450, device="cuda")
    pr, r1, r2 = p.astype(np.float64), np.zeros(450), np.zeros(450)
    for t in range(1, 6):
        grad = g.standard_normal(450).astype(np.float32)
        cg.casgd_adam_step(pd, _dev(grad), m1, m2, t, 1e-2)
        pr, r1, r2 = R.adam_step(pr, grad.astype(np.float64), r1, r2, t, 1e-2)
    assert np.allclose(pd.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_hess_diag_and_scaled_quantize(cg, fmt):
    p = dense_logreg(2000, 300, 5, var=1 / 300, noise_var=0.1, dtype=np.float32)
    code = {"f32": cg.F32, "bf16": cg.BF16}[fmt]
    d = np.exp(np.random.default_rng(1).uniform(-1, 1, 300)).astype(np.float32)
    src = _dev(p.X)
    stored, sc = cg.casgd_quantize_scaled(src, _dev(d), code)
    Xs = cg.dense_matrix(stored, sc, n=300)
    # the oracle's exact stored values of the scaled matrix
    scaled = (p.X * d[None, :]).astype(np.float32)
    _, _, exact = R.quantize(scaled, fmt)
    x = (np.random.default_rng(2).standard_normal(300) * 0.3).astype(np.float32)
    h = cg.casgd_hess_diag(Xs, _dev(x), 1e-3).cpu().numpy()
    ref = R.hess_diag(exact, x, 1e-3)
    assert np.allclose(h, ref, rtol=1e-4)


def test_feature_norm_apply_and_jacobi_target_vs_oracle(cg):
    g = np.random.default_rng(4)
    st = (np.abs(g.standard_normal((3000, 4))) * [1, 10, 0.1, 3]).astype(np.float32)
    norm = cg.casgd_mlp_feature_norm(_dev(st)).cpu().numpy()
    mu, sd = R.feature_norm(st)
    assert np.allclose(norm[:4], mu, rtol=1e-6, atol=1e-7)
    assert np.allclose(norm[4:], sd, rtol=1e-6)

    o = (g.standard_normal((2500, 2)) * [3.0, 0.5]).astype(np.float32)
    o[7, 0] = 60.0   # clipped
    q, eta = cg.casgd_mlp_apply(_dev(o))
    rq, reta = R.mlp_apply(o)
    assert np.allclose(q.cpu().numpy(), rq, rtol=1e-6)
    assert np.isclose(float(eta), reta, rtol=1e-6)

    h = np.exp(g.uniform(-5, 5, 2049)).astype(np.float32)
    t_d, q = cg.casgd_jacobi_target(_dev(h))
    rt, rq = R.jacobi_target(h)
    assert np.allclose(t_d.cpu().numpy(), rt, atol=2e-6)
    assert np.allclose(q.cpu().numpy(), rq, rtol=2e-6)
